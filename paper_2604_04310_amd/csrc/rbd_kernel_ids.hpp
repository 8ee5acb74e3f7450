// Every kernel a topology provides, in one list shared by the ahead-of-time
// build (which takes each kernel's address) and the runtime compiler (which
// names each kernel to hiprtc): id, compilation part, and the kernel template
// instantiated for the topology's tree type TP. The parts group kernels that
// compile together ahead of time: 1 kinematics, inverse dynamics and mass
// matrix; 2 forward dynamics and the packed forward / inverse dynamics
// launches; 3 the adjoint and its packed launch; 4 the articulated-body
// algorithm; 5 the external-force variants; 6 the forward-mode derivative;
// 7 the controllers; 8 the derivatives with external forces.
#pragma once

#define RBD_KERNELS(X)                                    \
  X(KID_FK, 1, k_fk<TP>)                                  \
  X(KID_JACOBIAN, 1, k_jacobian<TP>)                      \
  X(KID_RNEA_BIAS, 1, k_rnea<TP, false, false, false>)    \
  X(KID_RNEA, 1, k_rnea<TP, true, false, false>)          \
  X(KID_RNEA_BIAS_PRE, 1, k_rnea<TP, false, false, true>) \
  X(KID_RNEA_PRE, 1, k_rnea<TP, true, false, true>)       \
  X(KID_CRBA, 1, k_crba<TP>)                              \
  X(KID_FWD_DYN, 2, k_fwd_dyn<TP, false, false>)          \
  X(KID_FWD_DYN_PRE, 2, k_fwd_dyn<TP, true, false>)       \
  X(KID_PACKED_FWD_DYN, 2, k_packed<TP, 0>)               \
  X(KID_PACKED_RNEA, 2, k_packed<TP, 1>)                  \
  X(KID_VJP_TAU, 3, k_fwd_dyn_vjp<TP, 0>)                 \
  X(KID_VJP_REGS, 3, k_fwd_dyn_vjp<TP, 1>)                \
  X(KID_VJP_PARK, 3, k_fwd_dyn_vjp<TP, 2>)                \
  X(KID_PACKED_VJP, 3, k_packed<TP, 2>)                   \
  X(KID_ABA, 4, k_aba<TP, false, false>)                  \
  X(KID_ABA_PRE, 4, k_aba<TP, true, false>)               \
  X(KID_RNEA_BIAS_EXT, 5, k_rnea<TP, false, true, false>) \
  X(KID_RNEA_EXT, 5, k_rnea<TP, true, true, false>)       \
  X(KID_FWD_DYN_EXT, 5, k_fwd_dyn<TP, false, true>)       \
  X(KID_FWD_DYN_PRE_EXT, 5, k_fwd_dyn<TP, true, true>)    \
  X(KID_ABA_EXT, 5, k_aba<TP, false, true>)               \
  X(KID_ABA_PRE_EXT, 5, k_aba<TP, true, true>)            \
  X(KID_JVP, 6, k_fwd_dyn_jvp<TP>)                        \
  X(KID_DIFF_IK, 7, k_diff_ik<TP>)                        \
  X(KID_OSC, 7, k_osc<TP>)                                \
  X(KID_VJP_EXT_REGS, 8, k_fwd_dyn_vjp<TP, 1, true>)      \
  X(KID_VJP_EXT_PARK, 8, k_fwd_dyn_vjp<TP, 2, true>)      \
  X(KID_JVP_EXT, 8, k_fwd_dyn_jvp<TP, true>)            \
  X(KID_VJP_LDS, 3, k_fwd_dyn_vjp<TP, 3>)                 \
  X(KID_VJP_EXT_LDS, 8, k_fwd_dyn_vjp<TP, 3, true>)       \
  X(KID_JVP_SPLIT, 6, k_fwd_dyn_jvp_split<TP>)            \
  X(KID_JVP_EXT_SPLIT, 8, k_fwd_dyn_jvp_split<TP, true>) \
  X(KID_RNEA_JVP, 6, k_rnea_jvp<TP>)                      \
  X(KID_RNEA_JVP_EXT, 8, k_rnea_jvp<TP, true>)           \
  X(KID_RNEA_JVP_PRE, 6, k_rnea_jvp<TP, false, true>)    \
  X(KID_RNEA_VJP, 3, k_rnea_vjp<TP>)                      \
  X(KID_RNEA_VJP_EXT, 8, k_rnea_vjp<TP, true>)            \
  X(KID_VJP_SPLIT, 3, k_fwd_dyn_vjp_split<TP>)            \
  X(KID_VJP_EXT_SPLIT, 8, k_fwd_dyn_vjp_split<TP, true>)

namespace rbd {

enum KernelId : int {
#define RBD_KID_ENUM(id, part, ...) id,
  RBD_KERNELS(RBD_KID_ENUM)
#undef RBD_KID_ENUM
  KID_COUNT
};

constexpr int kParts = 8;

}  // namespace rbd
