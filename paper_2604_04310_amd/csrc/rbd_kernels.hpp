// HIP kernels for gfx950, templated on the compiled tree type, and the host
// launch wrappers each topology's translation unit instantiates. The per-lane
// algorithms live in rbd_lane.hpp.
#pragma once

#include <hip/hip_runtime.h>

#include "rbd_internal.hpp"
#include "rbd_lane.hpp"

namespace rbd {

constexpr int kBlock = 256;

RBD_DI int64_t lane_id() { return (int64_t)blockIdx.x * blockDim.x + threadIdx.x; }

template <class TP>
__global__ __launch_bounds__(kBlock) void k_fk(const float* __restrict__ tab, int64_t batch, int64_t ld,
                                               const float* __restrict__ q, float* __restrict__ T) {
  const int64_t b = lane_id();
  if (b >= batch) return;
  fk_lane<TP>(tab, In{q + b, ld}, Out{T + b, ld});
}

template <class TP>
__global__ __launch_bounds__(kBlock) void k_jacobian(const float* __restrict__ tab, int64_t batch, int64_t ld,
                                                     const float* __restrict__ q, JacSlots js,
                                                     float* __restrict__ J) {
  const int64_t b = lane_id();
  if (b >= batch) return;
  jac_lane<TP>(tab, In{q + b, ld}, js, J + b, ld);
}

template <class TP, bool HAS_QDD>
__global__ __launch_bounds__(kBlock) void k_rnea(const float* __restrict__ tab, int64_t batch, int64_t ld,
                                                 const float* __restrict__ q, const float* __restrict__ qd,
                                                 const float* __restrict__ qdd, float* __restrict__ tau) {
  const int64_t b = lane_id();
  if (b >= batch) return;
  rnea_lane<TP, HAS_QDD>(tab, In{q + b, ld}, In{qd + b, ld}, In{HAS_QDD ? qdd + b : q + b, ld}, Out{tau + b, ld});
}

template <class TP>
__global__ __launch_bounds__(kBlock) void k_crba(const float* __restrict__ tab, int64_t batch, int64_t ld,
                                                 const float* __restrict__ q, float* __restrict__ M) {
  const int64_t b = lane_id();
  if (b >= batch) return;
  crba_lane<TP>(tab, In{q + b, ld}, M + b, ld);
}

struct RhsTau {
  In tau;
  RBD_DI float operator()(int, int k) const { return tau(k); }
};
struct SinkOut {
  Out x;
  RBD_DI void operator()(int, int k, float v) const { x(k, v); }
};

template <class TP>
__global__ __launch_bounds__(kBlock) void k_fwd_dyn(const float* __restrict__ tab, int64_t batch, int64_t ld,
                                                    const float* __restrict__ q, const float* __restrict__ qd,
                                                    const float* __restrict__ tau, float* __restrict__ qdd) {
  const int64_t b = lane_id();
  if (b >= batch) return;
  fwd_dyn_lane<TP, 1>(tab, In{q + b, ld}, In{qd + b, ld}, RhsTau{In{tau + b, ld}}, SinkOut{Out{qdd + b, ld}});
}

// ---- fwd_dyn adjoint: solve M [qdd, lam] = [tau - h, gbar] with one factor,
// write g_tau = lam, then run the inverse-dynamics adjoint at (q, qd, qdd).
struct RhsTwo {
  In tau, gbar;
  RBD_DI float operator()(int r, int k) const { return r == 0 ? tau(k) : gbar(k); }
};
struct SinkTwo {
  float* qdd;
  float* lam;
  RBD_DI void operator()(int r, int k, float v) const {
    if (r == 0) qdd[k] = v; else lam[k] = v;
  }
};
struct RegView {
  const float* x;
  RBD_DI float operator()(int k) const { return x[k]; }
};
struct OutOpt {
  float* __restrict__ p;
  int64_t ld;
  RBD_DI void operator()(int c, float v) const {
    if (p) p[c * ld] = v;
  }
};

template <class TP, bool ADJ>
RBD_DI void vjp_lane(const float* __restrict__ tab, const In& q, const In& qd, const In& tau, const In& gqdd,
                     const OutOpt& gq, const OutOpt& gqd, const OutOpt& gtau) {
  constexpr int NV = TP::NV;
  float qddv[NV], lam[NV];
  fwd_dyn_lane<TP, 2>(tab, q, qd, RhsTwo{tau, gqdd}, SinkTwo{qddv, lam});
  sfor<0, NV>([&](auto K_) __attribute__((always_inline)) {
    constexpr int K = decltype(K_)::value;
    gtau(K, lam[K]);
  });
  if constexpr (ADJ) id_adjoint_lane<TP>(tab, q, qd, RegView{qddv}, RegView{lam}, gq, gqd);
}

template <class TP, bool ADJ>
__global__ __launch_bounds__(kBlock) void k_fwd_dyn_vjp(const float* __restrict__ tab, int64_t batch, int64_t ld,
                                                        const float* __restrict__ q, const float* __restrict__ qd,
                                                        const float* __restrict__ tau,
                                                        const float* __restrict__ gqdd, float* __restrict__ gq,
                                                        float* __restrict__ gqd, float* __restrict__ gtau) {
  const int64_t b = lane_id();
  if (b >= batch) return;
  vjp_lane<TP, ADJ>(tab, In{q + b, ld}, In{qd + b, ld}, In{tau + b, ld}, In{gqdd + b, ld},
                    OutOpt{gq ? gq + b : nullptr, ld}, OutOpt{gqd ? gqd + b : nullptr, ld},
                    OutOpt{gtau ? gtau + b : nullptr, ld});
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
    const In q{R.in[0] + i * NQ, 1}, qd{R.in[1] + i * NV, 1}, x2{R.in[2] + i * NV, 1};
    if constexpr (OP == RBD_OP_FWD_DYN) {
      fwd_dyn_lane<TP, 1>(tab, q, qd, RhsTau{x2}, SinkOut{Out{R.out[0] + i * NV, 1}});
    } else if constexpr (OP == RBD_OP_RNEA) {
      rnea_lane<TP, true>(tab, q, qd, x2, Out{R.out[0] + i * NV, 1});
    } else {
      vjp_lane<TP, true>(tab, q, qd, x2, In{R.in[3] + i * NV, 1}, OutOpt{R.out[0] + i * NQ, 1},
                         OutOpt{R.out[1] + i * NV, 1}, OutOpt{R.out[2] + i * NV, 1});
    }
  }
}

// ------------------------------------------------------------------ launchers
static inline int grid_for(int64_t batch) { return (int)((batch + kBlock - 1) / kBlock); }

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
  static rbd_status rnea(const float* tab, int64_t batch, int64_t ld, const float* q, const float* qd,
                         const float* qdd, float* tau, hipStream_t s) {
    if (qdd)
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_rnea<TP, true>), dim3(grid_for(batch)), dim3(kBlock), 0, s, tab, batch,
                         ld, q, qd, qdd, tau);
    else
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_rnea<TP, false>), dim3(grid_for(batch)), dim3(kBlock), 0, s, tab, batch,
                         ld, q, qd, qdd, tau);
    return check_launch("rbd_rnea");
  }
  static rbd_status crba(const float* tab, int64_t batch, int64_t ld, const float* q, float* M, hipStream_t s) {
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_crba<TP>), dim3(grid_for(batch)), dim3(kBlock), 0, s, tab, batch, ld, q,
                       M);
    return check_launch("rbd_crba");
  }
  static rbd_status fwd_dyn(const float* tab, int64_t batch, int64_t ld, const float* q, const float* qd,
                            const float* tau, float* qdd, hipStream_t s) {
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_fwd_dyn<TP>), dim3(grid_for(batch)), dim3(kBlock), 0, s, tab, batch, ld,
                       q, qd, tau, qdd);
    return check_launch("rbd_fwd_dyn");
  }
  static rbd_status vjp(const float* tab, int64_t batch, int64_t ld, const float* q, const float* qd,
                        const float* tau, const float* gqdd, float* gq, float* gqd, float* gtau, hipStream_t s) {
    if (gq || gqd)
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_fwd_dyn_vjp<TP, true>), dim3(grid_for(batch)), dim3(kBlock), 0, s, tab,
                         batch, ld, q, qd, tau, gqdd, gq, gqd, gtau);
    else
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_fwd_dyn_vjp<TP, false>), dim3(grid_for(batch)), dim3(kBlock), 0, s, tab,
                         batch, ld, q, qd, tau, gqdd, gq, gqd, gtau);
    return check_launch("rbd_fwd_dyn_vjp");
  }
  static rbd_status packed(int op, const float* tab, const void* table, int grid, hipStream_t s) {
    const uint8_t* t = static_cast<const uint8_t*>(table);
    switch (op) {
      case RBD_OP_FWD_DYN:
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_packed<TP, RBD_OP_FWD_DYN>), dim3(grid), dim3(kBlock), 0, s, tab, t);
        break;
      case RBD_OP_RNEA:
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_packed<TP, RBD_OP_RNEA>), dim3(grid), dim3(kBlock), 0, s, tab, t);
        break;
      default:
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_packed<TP, RBD_OP_FWD_DYN_VJP>), dim3(grid), dim3(kBlock), 0, s, tab,
                           t);
        break;
    }
    return check_launch("packed launch");
  }
  static LaunchTable table() {
    return LaunchTable{&Launch::fk, &Launch::jacobian, &Launch::rnea, &Launch::crba,
                       &Launch::fwd_dyn, &Launch::vjp, &Launch::packed};
  }
};

}  // namespace rbd
