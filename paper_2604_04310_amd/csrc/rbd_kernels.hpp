// HIP kernels for gfx950, templated on the tree type. Device code only, with
// no host headers: the ahead-of-time build instantiates it per compiled
// topology (rbd_kern_topo.hip) and the runtime compiler per new topology
// (rbd_jit.cpp), from the same text. The per-lane algorithms live in
// rbd_lane.hpp; kernel ids and launch shapes are chosen on the host
// (rbd_dispatch.cpp).
#pragma once

#include "rbd_lane.hpp"
#include "rbd_shared.hpp"

namespace rbd {

RBD_DI uint32_t lane_id() { return blockIdx.x * blockDim.x + threadIdx.x; }

// The same pointer value, hidden from the optimiser (an empty asm on its
// scalar register, no instruction). A kernel that runs several sweeps gives
// each its own copies of the table and input pointers and of the row stride,
// so model constants, inputs, row addresses and what is computed from them
// (joint sines and cosines) are reloaded and recomputed in each sweep instead
// of being held in registers across all of them.
// The asm operand keeps the pointer's address space (global for inputs,
// constant for the model table), so loads through the copy stay global loads
// with a scalar base, and table reads stay scalar loads.
RBD_DI const float* opaque(const float* p) {
  auto g = (const __attribute__((address_space(1))) float*)p;
  asm volatile("" : "+s"(g));
  return (const float*)g;
}
RBD_DI const float* opaque_table(const float* p) {
  auto c = (const __attribute__((address_space(4))) float*)p;
  asm volatile("" : "+s"(c));
  return (const float*)c;
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
// Loads entries 0..n-1 of input views into registers.
template <int n, class A>
RBD_DI void preload_inputs(float (&x)[n], const A& a) {
  sfor<0, n>([&](auto K_) __attribute__((always_inline)) { x[decltype(K_)::value] = a(decltype(K_)::value); });
}
template <int n, class A, class B>
RBD_DI void preload_inputs(float (&x)[n], float (&y)[n], const A& a, const B& b) {
  sfor<0, n>([&](auto K_) __attribute__((always_inline)) {
    constexpr int K = decltype(K_)::value;
    x[K] = a(K);
    y[K] = b(K);
  });
}

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
// A per-lane row parked in LDS: entry c of lane l of a wave at
// p[c * 64 + l] (consecutive lanes in consecutive banks; the entry offset is
// a compile-time immediate).
struct LdsRow {
  float* p;
  RBD_DI void operator()(int c, float v) const { p[c * kTileLanes] = v; }
  struct In {
    const float* p;
    RBD_DI float operator()(int c) const { return p[c * kTileLanes]; }
  };
};

template <class TP, bool ADJ, class QI, class X, class GQ, class GQD, class GT, class FX = NoFext, class GF = NoGF>
RBD_DI void vjp_lane(const float* __restrict__ tab, const QI& q, const X& qd, const X& tau, const X& gqdd,
                     const GQ& gq, const GQD& gqd, const GT& gtau, const FX& fx = FX{}, const GF& gf = GF{}) {
  constexpr int NV = TP::NV;
  float qddv[NV], lam[NV];
  fwd_dyn_lane<TP, 2>(tab, q, qd, RhsTwo<X>{tau, gqdd}, SinkRegs{qddv, lam}, fx);
  sfor<0, NV>([&](auto K_) __attribute__((always_inline)) {
    constexpr int K = decltype(K_)::value;
    gtau(K, lam[K]);
  });
  if constexpr (ADJ) id_adjoint_lane<TP>(tab, q, qd, RegView{qddv}, RegView{lam}, gq, gqd, fx, gf);
}

// q-double-dot parked in g_qd and lam in g_tau between the solve and the
// adjoint sweep, instead of 2 nv registers held across it. Every element is
// read by its body's forward step before that body's backward step
// overwrites g_qd.
template <class TP, class QI, class X, class GQ, class P, class FX = NoFext, class GF = NoGF>
RBD_DI void vjp_lane_parked(const float* __restrict__ tab, const QI& q, const X& qd, const X& tau, const X& gqdd,
                            const GQ& gq, const P& gqd_out, const P& gtau_out, const typename P::In& gqd_in,
                            const typename P::In& gtau_in, const FX& fx = FX{}, const GF& gf = GF{}) {
  fwd_dyn_lane<TP, 2>(tab, q, qd, RhsTwo<X>{tau, gqdd}, SinkTwo<P>{gqd_out, gtau_out}, fx);
  id_adjoint_lane<TP>(tab, q, qd, gqd_in, gtau_in, gq, gqd_out, fx, gf);
}

struct RowAlias {
  GlobalF* p;
  RBD_DI RowAlias(float* q) : p((GlobalF*)q) {}
  RBD_DI void operator()(int c, float v) const { p[c] = v; }
  struct In {
    const GlobalF* p;
    RBD_DI In(const float* q) : p((const GlobalF*)q) {}
    RBD_DI float operator()(int c) const { return p[c]; }
  };
};

// MODE 0: g_tau only; 1: adjoint with q-double-dot and lam in registers (some
// output absent); 2: adjoint with both parked in g_qd and g_tau (both
// requested); 3 (large trees, any outputs): both parked in LDS (dynamic shared
// memory, 2 NV floats per lane), the adjoint on fresh views. EXT (modes 1 to
// 3): external forces fext (nullable: zero) in the dynamics and the force
// cotangent g_fext (nullable).
template <class TP, int MODE, bool EXT = false>
__global__ __launch_bounds__(kBlock) void k_fwd_dyn_vjp(const float* __restrict__ tab, int64_t batch, int64_t ld,
                                                        const float* __restrict__ q, const float* __restrict__ qd,
                                                        const float* __restrict__ tau,
                                                        const float* __restrict__ gqdd, float* gq, float* gqd,
                                                        float* gtau, const float* __restrict__ fext, float* gfext) {
  static_assert(!EXT || MODE >= 1, "external forces: modes 1 to 3");
  RBD_LANE_IO(TP);
  const uint32_t b = lane_id();
  if (b >= batch) return;
  const In qi{q, ld, b}, qdi{qd, ld, b}, ti{tau, ld, b}, gi{gqdd, ld, b};
  const OutOpt<OutAlias> gqo{OutAlias{gq, ld, b}, gq != nullptr};
  // the external-force views (nothing without EXT)
  auto fx_view = [&](const float* p, int64_t l) __attribute__((always_inline)) {
    if constexpr (EXT) return FextOpt{{p, l, b}};
    else return NoFext{};
  };
  auto gf_view = [&](int64_t l) __attribute__((always_inline)) {
    if constexpr (EXT) return GFOut{{gfext, l, b}};
    else return NoGF{};
  };
  if constexpr (MODE == 3) {
    // the two sweeps, the second on fresh views (its own table and input
    // pointers and row stride): a large tree's first sweep uses every
    // register, and values kept for the second one spill (measured: 1028 ->
    // 400 B/lane of scratch, 126 -> 108 us for the humanoid). Each wave parks
    // in its region of the block's dynamic LDS: [qdd rows | lam rows].
    extern __shared__ float lds_park[];
    constexpr int NV = TP::NV;
    float* const w = lds_park + (threadIdx.x / kTileLanes) * (2 * NV * kTileLanes) + (threadIdx.x % kTileLanes);
    fwd_dyn_lane<TP, 2>(tab, qi, qdi, RhsTwo<In>{ti, gi}, SinkTwo<LdsRow>{LdsRow{w}, LdsRow{w + NV * kTileLanes}},
                        fx_view(fext, ld));
    if (gtau) {
      sfor<0, NV>([&](auto K_) __attribute__((always_inline)) {
        constexpr int K = decltype(K_)::value;
        Out{gtau, ld, b}(K, w[(NV + K) * kTileLanes]);
      });
    }
    sweep_boundary();
    const int64_t l2 = opaque(ld);
    // (issuing this sweep's q and qd loads at its start cut the spill from 536
    // to 24 B/lane but measured 79.2 against 77.0 us for the humanoid at 32768)
    id_adjoint_lane<TP>(opaque_table(tab), In{opaque(q), l2, b}, In{opaque(qd), l2, b}, LdsRow::In{w},
                        LdsRow::In{w + NV * kTileLanes}, OutOpt<OutAlias>{OutAlias{gq, l2, b}, gq != nullptr},
                        OutOpt<OutAlias>{OutAlias{gqd, l2, b}, gqd != nullptr}, fx_view(opaque(fext), l2),
                        gf_view(l2));
  } else if constexpr (MODE == 2) {
    const OutAliasP pd{{gqd, ld, b}}, pt{{gtau, ld, b}};
    vjp_lane_parked<TP>(tab, qi, qdi, ti, gi, gqo, pd, pt, InAlias{gqd, ld, b}, InAlias{gtau, ld, b},
                        fx_view(fext, ld), gf_view(ld));
  } else {
    vjp_lane<TP, MODE == 1>(tab, qi, qdi, ti, gi, gqo, OutOpt<OutAlias>{OutAlias{gqd, ld, b}, gqd != nullptr},
                            OutOpt<OutAlias>{OutAlias{gtau, ld, b}, gtau != nullptr}, fx_view(fext, ld),
                            gf_view(ld));
  }
}

// ---- the adjoint on two waves per 64 instances (a block of 128 lanes), for
// large trees at batches small enough that one wave per 64 instances leaves
// SIMDs idle: wave 0 solves for qdd (the fused sweep) while wave 1 factors M
// on its own and solves lam = M^-1 g_qdd (the bias-free sweep; g_tau = lam).
// Nothing but qdd and lam crosses the block's one barrier, parked in LDS
// ([qdd rows | lam rows], 64 lanes each); then wave 0 runs the adjoint sweep
// on fresh views. Every lane of the block reaches the barrier.
template <class TP, bool EXT = false>
__global__ __launch_bounds__(2 * kTileLanes) void k_fwd_dyn_vjp_split(
    const float* __restrict__ tab, int64_t batch, int64_t ld, const float* __restrict__ q,
    const float* __restrict__ qd, const float* __restrict__ tau, const float* __restrict__ gqdd, float* gq,
    float* gqd, float* gtau, const float* __restrict__ fext, float* gfext) {
  RBD_LANE_IO(TP);
  constexpr int NQ = TP::NQ, NV = TP::NV;
  extern __shared__ float lds_vjp[];
  const uint32_t lane = threadIdx.x % kTileLanes;
  const bool solver = threadIdx.x >= kTileLanes;
  const uint32_t b = blockIdx.x * kTileLanes + lane;
  const bool valid = b < batch;
  float* const qpark = lds_vjp + lane;
  float* const lpark = lds_vjp + NV * kTileLanes + lane;
  auto fx_view = [&](const float* p, int64_t l) __attribute__((always_inline)) {
    if constexpr (EXT) return FextOpt{{p, l, b}};
    else return NoFext{};
  };
  auto gf_view = [&](int64_t l) __attribute__((always_inline)) {
    if constexpr (EXT) return GFOut{{gfext, l, b}};
    else return NoGF{};
  };
  if (!solver) {
    if (valid) {
      if constexpr (EXT) {
        fwd_dyn_lane<TP, 1>(tab, In{q, ld, b}, In{qd, ld, b}, RhsOne<In>{In{tau, ld, b}},
                            SinkOne<LdsRow>{LdsRow{qpark}}, fx_view(fext, ld));
      } else {
        // every input load at entry, as in k_fwd_dyn for large trees
        float qv[NQ], qdv[NV], tv[NV];
        preload_inputs<NQ>(qv, In{q, ld, b});
        preload_inputs<NV>(qdv, tv, In{qd, ld, b}, In{tau, ld, b});
        fwd_dyn_lane<TP, 1>(tab, RegView{qv}, RegView{qdv}, RhsOne<RegView>{RegView{tv}},
                            SinkOne<LdsRow>{LdsRow{qpark}});
      }
    }
  } else if (valid) {
    fwd_dyn_lane<TP, 1, In, In, RhsOne<In>, SinkOne<LdsRow>, NoFext, false>(
        tab, In{q, ld, b}, In{qd, ld, b}, RhsOne<In>{In{gqdd, ld, b}}, SinkOne<LdsRow>{LdsRow{lpark}});
    if (gtau) {
      sfor<0, NV>([&](auto K_) __attribute__((always_inline)) {
        constexpr int K = decltype(K_)::value;
        Out{gtau, ld, b}(K, lpark[K * kTileLanes]);
      });
    }
  }
  __syncthreads();
  if (!solver && valid) {
    sweep_boundary();
    const int64_t l2 = opaque(ld);
    id_adjoint_lane<TP>(opaque_table(tab), In{opaque(q), l2, b}, In{opaque(qd), l2, b}, LdsRow::In{qpark},
                        LdsRow::In{lpark}, OutOpt<OutAlias>{OutAlias{gq, l2, b}, gq != nullptr},
                        OutOpt<OutAlias>{OutAlias{gqd, l2, b}, gqd != nullptr}, fx_view(opaque(fext), l2),
                        gf_view(l2));
  }
}

// ---- fwd_dyn tangent, three sweeps of one lane: qdd by the fused solve
// (parked in the qdd output when one is given, else in dqdd), the tangent of
// inverse dynamics writing dtau - d(ID) into dqdd, and the solve with M in
// place (each right-hand-side entry is read when its subtree closes, every
// result written after the sweep). Neither output is restrict-qualified, so
// loads of parked values stay ordered with the stores.
// EXT: external forces fext and their tangent dfext (each nullable: zero).
template <class TP, bool EXT = false>
__global__ __launch_bounds__(kBlock) void k_fwd_dyn_jvp(const float* __restrict__ tab, int64_t batch, int64_t ld,
                                                        const float* __restrict__ q, const float* __restrict__ qd,
                                                        const float* __restrict__ tau, const float* __restrict__ dq,
                                                        const float* __restrict__ dqd,
                                                        const float* __restrict__ dtau, float* qdd, float* dqdd,
                                                        const float* __restrict__ fext,
                                                        const float* __restrict__ dfext) {
  RBD_LANE_IO(TP);
  const uint32_t b = lane_id();
  if (b >= batch) return;
  float* park = qdd ? qdd : dqdd;
  auto fx_view = [&](const float* p, int64_t l) __attribute__((always_inline)) {
    if constexpr (EXT) return FextOpt{{p, l, b}};
    else return NoFext{};
  };
  fwd_dyn_lane<TP, 1>(tab, In{q, ld, b}, In{qd, ld, b}, RhsOne<In>{In{tau, ld, b}},
                      SinkOne<OutAlias>{OutAlias{park, ld, b}}, fx_view(fext, ld));
  // a large tree gives each sweep fresh views (see k_fwd_dyn_vjp)
  constexpr bool kFresh = TP::NV > 16;
  auto view = [](auto x) __attribute__((always_inline)) {
    if constexpr (kFresh) return opaque(x);
    else return x;
  };
  auto view_table = [](const float* x) __attribute__((always_inline)) {
    if constexpr (kFresh) return opaque_table(x);
    else return x;
  };
  const int64_t ld2 = view(ld);
  if constexpr (kFresh && !EXT) {
    // every input load of the tangent sweep issued at its start, as in k_rnea_jvp
    constexpr int NQ = TP::NQ, NV = TP::NV;
    float qv[NQ], qdv[NV], dqv[NQ], dqdv[NV], dtv[NV];
    preload_inputs<NQ>(qv, dqv, In{view(q), ld2, b}, In{dq, ld2, b});
    preload_inputs<NV>(qdv, dqdv, In{view(qd), ld2, b}, In{dqd, ld2, b});
    preload_inputs<NV>(dtv, In{dtau, ld2, b});
    id_tangent_lane<TP>(view_table(tab), RegView{qv}, RegView{qdv}, InAlias{park, ld2, b}, RegView{dqv},
                        RegView{dqdv}, RegView{dtv}, OutAlias{dqdd, ld2, b});
  } else {
    id_tangent_lane<TP>(view_table(tab), In{view(q), ld2, b}, In{view(qd), ld2, b}, InAlias{park, ld2, b},
                        In{dq, ld2, b}, In{dqd, ld2, b}, In{dtau, ld2, b}, OutAlias{dqdd, ld2, b},
                        fx_view(fext, ld2), fx_view(dfext, ld2));
  }
  const int64_t ld3 = view(ld2);
  fwd_dyn_lane<TP, 1, In, In, RhsOne<InAlias>, SinkOne<OutAlias>, NoFext, false>(
      view_table(tab), In{view(q), ld3, b}, In{qd, ld3, b}, RhsOne<InAlias>{InAlias{dqdd, ld3, b}},
      SinkOne<OutAlias>{OutAlias{dqdd, ld3, b}});
}

// ---- the same tangent on two waves per 64 instances (a block of 128 lanes),
// for batches small enough that one wave per 64 instances leaves SIMDs idle:
// wave 0 runs the fused solve for qdd and the tangent of inverse dynamics and
// hands the right-hand side to wave 1 through LDS; wave 1 factors M in the
// meantime, then solves with it. Dynamic LDS per block: [rhs rows | qdd rows],
// 64 lanes each. Every lane of the block reaches the one barrier.
template <class TP, bool EXT = false>
__global__ __launch_bounds__(2 * kTileLanes) void k_fwd_dyn_jvp_split(
    const float* __restrict__ tab, int64_t batch, int64_t ld, const float* __restrict__ q,
    const float* __restrict__ qd, const float* __restrict__ tau, const float* __restrict__ dq,
    const float* __restrict__ dqd, const float* __restrict__ dtau, float* qdd, float* dqdd,
    const float* __restrict__ fext, const float* __restrict__ dfext) {
  RBD_LANE_IO(TP);
  constexpr int NV = TP::NV;
  extern __shared__ float lds_jvp[];
  const uint32_t lane = threadIdx.x % kTileLanes;
  const bool solver = threadIdx.x >= kTileLanes;
  const uint32_t b = blockIdx.x * kTileLanes + lane;
  const bool valid = b < batch;
  float* const rhs = lds_jvp + lane;
  float* const qpark = lds_jvp + NV * kTileLanes + lane;
  auto fx_view = [&](const float* p, int64_t l) __attribute__((always_inline)) {
    if constexpr (EXT) return FextOpt{{p, l, b}};
    else return NoFext{};
  };
  Ltl<TP, 1> F;
  if (!solver) {
    if (valid) {
      fwd_dyn_lane<TP, 1>(tab, In{q, ld, b}, In{qd, ld, b}, RhsOne<In>{In{tau, ld, b}},
                          SinkOne<LdsRow>{LdsRow{qpark}}, fx_view(fext, ld));
      if (qdd) {
        sfor<0, NV>([&](auto K_) __attribute__((always_inline)) {
          constexpr int K = decltype(K_)::value;
          Out{qdd, ld, b}(K, qpark[K * kTileLanes]);
        });
      }
      sweep_boundary();
      const int64_t l2 = opaque(ld);
      if constexpr (!EXT) {
        // every input load of the tangent sweep issued at its start, as in k_rnea_jvp
        constexpr int NQ = TP::NQ;
        float qv[NQ], qdv[NV], dqv[NQ], dqdv[NV], dtv[NV];
        preload_inputs<NQ>(qv, dqv, In{opaque(q), l2, b}, In{dq, l2, b});
        preload_inputs<NV>(qdv, dqdv, In{opaque(qd), l2, b}, In{dqd, l2, b});
        preload_inputs<NV>(dtv, In{dtau, l2, b});
        id_tangent_lane<TP>(opaque_table(tab), RegView{qv}, RegView{qdv}, LdsRow::In{qpark}, RegView{dqv},
                            RegView{dqdv}, RegView{dtv}, LdsRow{rhs});
      } else {
        id_tangent_lane<TP>(opaque_table(tab), In{opaque(q), l2, b}, In{opaque(qd), l2, b}, LdsRow::In{qpark},
                            In{dq, l2, b}, In{dqd, l2, b}, In{dtau, l2, b}, LdsRow{rhs}, fx_view(opaque(fext), l2),
                            fx_view(opaque(dfext), l2));
      }
    }
  } else if (valid) {
    ltl_factor_lane<TP>(tab, In{q, ld, b}, F);
  }
  __syncthreads();
  if (solver && valid) {
    ltl_solve_y<TP>(F, LdsRow::In{rhs});
    ltl_back<TP, 1>(F, [&](int, int k, float v) __attribute__((always_inline)) { Out{dqdd, ld, b}(k, v); });
  }
}

// ---- tangent of inverse dynamics, Eq. (1), along (dq, dqd, dqdd[, dF]): one
// sweep of id_tangent_lane with the acceleration tangent; the sweep writes
// 0 - d(ID), stored negated as d(ID) (both steps exact).
template <class V>
struct On : V {  // a view whose entries are used (kOn)
  static constexpr bool kOn = true;
};
template <class O>
struct Neg {  // an output written negated
  O o;
  static constexpr bool kOn = true;
  RBD_DI void operator()(int c, float v) const { o(c, -v); }
};

// PRE (no external forces): every input load is issued at entry, as in
// k_fwd_dyn.
template <class TP, bool EXT = false, bool PRE = false>
__global__ __launch_bounds__(kBlock) void k_rnea_jvp(const float* __restrict__ tab, int64_t batch, int64_t ld,
                                                     const float* __restrict__ q, const float* __restrict__ qd,
                                                     const float* __restrict__ qdd, const float* __restrict__ dq,
                                                     const float* __restrict__ dqd, const float* __restrict__ dqdd,
                                                     float* __restrict__ dtau, const float* __restrict__ fext,
                                                     const float* __restrict__ dfext) {
  RBD_LANE_IO(TP);
  const uint32_t b = lane_id();
  if (b >= batch) return;
  auto fx_view = [&](const float* p) __attribute__((always_inline)) {
    if constexpr (EXT) return FextOpt{{p, ld, b}};
    else return NoFext{};
  };
  if constexpr (PRE && !EXT) {
    constexpr int NQ = TP::NQ, NV = TP::NV;
    float qv[NQ], qdv[NV], qddv[NV], dqv[NQ], dqdv[NV], dqddv[NV];
    const In qi{q, ld, b}, qdi{qd, ld, b}, qddi{qdd, ld, b}, dqi{dq, ld, b}, dqdi{dqd, ld, b}, dqddi{dqdd, ld, b};
    sfor<0, NQ>([&](auto K_) __attribute__((always_inline)) {
      constexpr int K = decltype(K_)::value;
      qv[K] = qi(K);
      dqv[K] = dqi(K);
    });
    sfor<0, NV>([&](auto K_) __attribute__((always_inline)) {
      constexpr int K = decltype(K_)::value;
      qdv[K] = qdi(K);
      qddv[K] = qddi(K);
      dqdv[K] = dqdi(K);
      dqddv[K] = dqddi(K);
    });
    id_tangent_lane<TP>(tab, RegView{qv}, RegView{qdv}, RegView{qddv}, RegView{dqv}, RegView{dqdv}, NoFext{},
                        Neg<Out>{Out{dtau, ld, b}}, NoFext{}, NoFext{}, On<RegView>{RegView{dqddv}});
  } else {
    id_tangent_lane<TP>(tab, In{q, ld, b}, In{qd, ld, b}, In{qdd, ld, b}, In{dq, ld, b}, In{dqd, ld, b}, NoFext{},
                        Neg<Out>{Out{dtau, ld, b}}, fx_view(fext), fx_view(dfext), On<In>{In{dqdd, ld, b}});
  }
}

// ---- adjoint of inverse dynamics, Eq. (1), for the cotangent lam: one sweep
// of id_adjoint_lane at the given qdd. That sweep writes the cotangents of
// forward dynamics, -lam^T dID/d(q, qd) and J_i lam, which are stored negated
// (exact), and g_qdd = M lam. Every output may be absent (null).
template <class TP, bool EXT = false>
__global__ __launch_bounds__(kBlock) void k_rnea_vjp(const float* __restrict__ tab, int64_t batch, int64_t ld,
                                                     const float* __restrict__ q, const float* __restrict__ qd,
                                                     const float* __restrict__ qdd, const float* __restrict__ lam,
                                                     float* __restrict__ gq, float* __restrict__ gqd,
                                                     float* __restrict__ gqdd, const float* __restrict__ fext,
                                                     float* __restrict__ gfext) {
  RBD_LANE_IO(TP);
  const uint32_t b = lane_id();
  if (b >= batch) return;
  auto opt = [&](float* p) __attribute__((always_inline)) { return OutOpt<Out>{Out{p, ld, b}, p != nullptr}; };
  auto fx_view = [&]() __attribute__((always_inline)) {
    if constexpr (EXT) return FextOpt{{fext, ld, b}};
    else return NoFext{};
  };
  auto gf_view = [&]() __attribute__((always_inline)) {
    if constexpr (EXT) return Neg<GFOut>{GFOut{{gfext, ld, b}}};
    else return NoGF{};
  };
  if constexpr (TP::NV > 16 && !EXT) {
    // every input load issued at entry, as in k_rnea_jvp
    constexpr int NQ = TP::NQ, NV = TP::NV;
    float qv[NQ], qdv[NV], qddv[NV], lv[NV];
    preload_inputs<NQ>(qv, In{q, ld, b});
    preload_inputs<NV>(qdv, qddv, In{qd, ld, b}, In{qdd, ld, b});
    preload_inputs<NV>(lv, In{lam, ld, b});
    id_adjoint_lane<TP>(tab, RegView{qv}, RegView{qdv}, RegView{qddv}, RegView{lv}, Neg<OutOpt<Out>>{opt(gq)},
                        Neg<OutOpt<Out>>{opt(gqd)}, NoFext{}, NoGF{}, On<OutOpt<Out>>{opt(gqdd)});
  } else {
    id_adjoint_lane<TP>(tab, In{q, ld, b}, In{qd, ld, b}, In{qdd, ld, b}, In{lam, ld, b}, Neg<OutOpt<Out>>{opt(gq)},
                        Neg<OutOpt<Out>>{opt(gqd)}, fx_view(), gf_view(), On<OutOpt<Out>>{opt(gqdd)});
  }
}

// ---- controller workloads for one frame E: the last body (a leaf) ahead of
// time, any other body compiled at run time on its first use.
template <class TP, int E = TP::N - 1>
__global__ __launch_bounds__(kBlock) void k_diff_ik(const float* __restrict__ tab, int64_t batch, int64_t ld,
                                                    const float* __restrict__ q, const float* __restrict__ tgt,
                                                    float gain, float lam2, float* __restrict__ qd) {
  RBD_LANE_IO(TP);
  const uint32_t b = lane_id();
  if (b >= batch) return;
  diff_ik_lane<TP, E>(tab, In{q, ld, b}, In{tgt, ld, b}, gain, lam2, Out{qd, ld, b});
}

// Two sweeps (bias force with the null-space solve, then the task-space
// solve), the second on fresh views; the torques written by the first are read
// back by the second, so tau is not restrict-qualified. Inputs are loaded
// where they are used (preloading them, as k_fwd_dyn does for large trees,
// held 83 more registers and measured 99 us against 81 us for the humanoid at
// batch 65536 with the sweeps fused).
template <class TP, int E = TP::N - 1>
__global__ __launch_bounds__(kBlock) void k_osc(const float* __restrict__ tab, int64_t batch, int64_t ld,
                                                const float* __restrict__ q, const float* __restrict__ qd,
                                                const float* __restrict__ tgt, float kp, float kd, float kn,
                                                float* tau) {
  RBD_LANE_IO(TP);
  const uint32_t b = lane_id();
  if (b >= batch) return;
  float ypath[TP::NV], astar[6];
  osc_sweep_bias<TP, E>(tab, In{q, ld, b}, In{qd, ld, b}, In{tgt, ld, b}, kp, kd, kn, OutAlias{tau, ld, b}, ypath,
                        astar);
  sweep_boundary();
  // the second sweep on fresh views (see k_fwd_dyn_vjp)
  const int64_t l2 = opaque(ld);
  osc_sweep_task<TP, E>(opaque_table(tab), In{opaque(q), l2, b}, ypath, astar, OutAlias{tau, l2, b},
                        InAlias{tau, l2, b});
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
    if constexpr (OP == kOpFwdDyn) {
      fwd_dyn_lane<TP, 1>(tab, q, qd, RhsOne<InRow>{x2}, SinkOne<OutRow>{OutRow{R.out[0] + i * NV}});
    } else if constexpr (OP == kOpRnea) {
      rnea_lane<TP, true>(tab, q, qd, x2, OutRow{R.out[0] + i * NV});
    } else {
      float* gqd = R.out[1] + i * NV;
      float* gtau = R.out[2] + i * NV;
      if constexpr (NV > 16) {
        // the two sweeps on fresh views, as in k_fwd_dyn_vjp
        fwd_dyn_lane<TP, 2>(tab, q, qd, RhsTwo<InRow>{x2, InRow{R.in[3] + i * NV}},
                            SinkTwo<RowAlias>{RowAlias{gqd}, RowAlias{gtau}});
        sweep_boundary();
        id_adjoint_lane<TP>(opaque_table(tab), InRow{opaque(R.in[0]) + i * NQ}, InRow{opaque(R.in[1]) + i * NV},
                            RowAlias::In{gqd}, RowAlias::In{gtau}, OutRow{R.out[0] + i * NQ}, RowAlias{gqd});
      } else {
        vjp_lane_parked<TP>(tab, q, qd, x2, InRow{R.in[3] + i * NV}, OutRow{R.out[0] + i * NQ}, RowAlias{gqd},
                            RowAlias{gtau}, RowAlias::In{gqd}, RowAlias::In{gtau});
      }
    }
  }
}

}  // namespace rbd
