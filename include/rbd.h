/*
 * rbd.h - batched rigid-body kinematics and dynamics on one MI355X (gfx950).
 *
 * C ABI of librbd.so. Every hot entry point evaluates one operation for a
 * whole batch of robot states, one instance per GPU lane, in FP32.
 *
 * Operations (arxiv 2604.04310):
 *   rbd_fk           forward kinematics 0T_i(q) of every body (Sec. II)
 *   rbd_jacobian     world-aligned geometric Jacobians of chosen body frames
 *                    (Sec. IV, the library's analytical Jacobians)
 *   rbd_rnea         inverse dynamics tau = M qdd + c + g - J^T F_ext,
 *                    Eq. (1); with qdd == NULL the bias force h(q, qd) (Alg. 1)
 *   rbd_crba         joint-space mass matrix M(q) (Alg. 2)
 *   rbd_fwd_dyn      forward dynamics qdd = M^-1 (tau - h + J^T F_ext), Eq. (2), by a
 *                    per-instance Cholesky-type solve (Sec. VI-A, footnote)
 *   rbd_aba          the same forward dynamics by the articulated-body
 *                    algorithm, O(n), no mass matrix (Sec. II names it among
 *                    Featherstone's algorithms; Sec. VI-A, future work)
 *   rbd_fwd_dyn_jvp  forward-mode derivative of rbd_fwd_dyn (Sec. IV-A, Fig. 2)
 *   rbd_rnea_jvp     forward-mode derivative of rbd_rnea (Sec. IV-A, Fig. 2)
 *   rbd_rnea_vjp     reverse-mode derivative of rbd_rnea (Sec. I, AD)
 *   rbd_diff_ik      differential IK for an end effector (Sec. IV, Table II)
 *   rbd_osc          operational-space control torques (Sec. IV, Table II)
 *   rbd_fwd_dyn_vjp  reverse-mode derivative of rbd_fwd_dyn (Sec. I, AD)
 *   rbd_server_*     continuous-batching service for the above (host API)
 *
 * Conventions
 *   Bodies are numbered 0..n-1 with parent[i] < i (-1 = world), depth-first
 *   (every subtree is a contiguous range of bodies). Body 0 may be a free
 *   joint. A revolute body frame sits at origin p in its parent frame, is
 *   turned by the fixed rotation R and then by q about the unit axis.
 *   Generalised coordinates: revolute q, qd, qdd, tau are scalars. A free base
 *   has q = [p_world(3); quaternion w,x,y,z (4)], qd = [v; w] (the body-frame
 *   twist of the base origin, linear first), qdd its time derivative, and tau
 *   the body-frame wrench [force; moment]. Base rotation = Hamilton rotation of
 *   the quaternion divided by its squared norm. nq = n (+6 with a free base),
 *   nv = n (+5 with a free base).
 *   Gravity enters as a fictitious base acceleration -g, so tau contains the
 *   holding torque +g(q).
 *
 * Data layout of every batched array: device memory, FP32, structure of
 *   arrays. Element (coordinate c, instance b) lives at ptr[c * ld + b] with
 *   ld >= batch; 0 <= batch <= 2^30 instances per call (RBD_E_INVAL beyond).
 *   Inputs are never written. Outputs must not overlap inputs.
 *
 * Calls are asynchronous on the given HIP stream (0 = the null stream). They
 *   never allocate device memory and never synchronise. Argument errors are
 *   reported synchronously by the status code, with a message from
 *   rbd_last_error() (thread-local). A numerically failed instance (a
 *   non-positive pivot, a zero quaternion) yields NaN in that instance's
 *   outputs and never fails the call.
 */
#ifndef RBD_H
#define RBD_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RBD_OK = 0,
  RBD_E_INVAL = 1,       /* bad argument (message in rbd_last_error)          */
  RBD_E_NOMEM = 2,       /* device or host allocation failed                  */
  RBD_E_NODEVICE = 3,    /* no usable GPU, or the device id is out of range   */
  RBD_E_LAUNCH = 4,      /* a HIP call or kernel launch failed                */
  RBD_E_UNSUPPORTED = 5, /* valid model whose topology has no compiled kernel */
  RBD_E_TIMEOUT = 6,     /* rbd_server_wait: the request did not finish       */
  RBD_E_SHUTDOWN = 7,    /* rbd_server_*: the server is shutting down         */
  RBD_E_COMPILE = 8,     /* run-time compilation of a new topology failed     */
  RBD_E_CANCELLED = 9    /* rbd_server_*: the request was cancelled           */
} rbd_status;

typedef enum { RBD_JOINT_REVOLUTE = 0, RBD_JOINT_FREE = 1 } rbd_joint;

/* Kinematic tree description, host memory, FP64 (paper Sec. II: a kinematic
 * tree with generalised coordinates q). Copied by rbd_model_create; the caller
 * keeps ownership. */
typedef struct {
  int32_t n_bodies;          /* 1 .. 64                                        */
  const int32_t* parent;     /* [n]  parent[i] < i, -1 = world                 */
  const int32_t* joint_type; /* [n]  rbd_joint; FREE only for body 0           */
  const double* axis;        /* [n][3] joint axis in the joint frame (revolute;
                                normalised on creation, must be non-zero)      */
  const double* origin;      /* [n][12] fixed parent->joint transform: rotation
                                R row-major (9) then p (3); unused for FREE    */
  const double* mass;        /* [n]  > 0                                       */
  const double* com;         /* [n][3] centre of mass in the body frame        */
  const double* inertia;     /* [n][6] about the CoM in body axes:
                                xx yy zz xy xz yz; positive definite           */
  double gravity[3];         /* world gravity, e.g. {0, 0, -9.81}              */
} rbd_tree_desc;

typedef struct rbd_model rbd_model; /* opaque: device-resident tables */

/* Validate the tree, precompute FP32 tables and upload them to `device`.
 * Any valid tree is accepted (Sec. II: a robot is a kinematic tree). The
 * library carries kernels compiled ahead of time for a list of topologies
 * (chains of 1-8 joints, a free body, a 12-body floating tree and the 30-body
 * humanoid). For any other topology the same kernel templates are compiled
 * for the tree with hiprtc at run time, one kernel at a time, the first time
 * that kernel is launched on a device (so the first call of each operation on
 * a new topology is host-synchronous and takes seconds for small trees, up to
 * minutes for a 40-body tree; the first call must not be made during stream
 * capture; controller kernels of other frames, see rbd_osc, are compiled the
 * same way). Code objects are cached on disk and looked up in $RBD_JIT_CACHE
 * (if set), then in "_jit" beside librbd.so (code objects installed with the
 * library, see rbd_precompile_topology), then in $XDG_CACHE_HOME/rbd-jit or
 * ~/.cache/rbd-jit; new ones are written to $RBD_JIT_CACHE, else the user
 * cache. A kernel is loaded once per process and device and serves every
 * model of its topology. Compute calls on such a model can then also return
 * RBD_E_COMPILE (compilation failed; message in rbd_last_error).
 * Errors: RBD_E_INVAL (null pointer, n out of range, parent[i] >= i, a
 * subtree that is not a contiguous range, FREE joint not at body 0, unknown
 * joint type, zero axis, R not a rotation, mass <= 0, inertia not positive
 * definite or violating the triangle inequality), RBD_E_NODEVICE,
 * RBD_E_NOMEM.
 * device = -1 creates a host-only model: validated, with its tables on the
 * host and no kernels; compute calls on it return RBD_E_NODEVICE. It serves a
 * server with the host executor (scheduling without a GPU, see below). */
rbd_status rbd_model_create(const rbd_tree_desc* desc, int device, rbd_model** out);
rbd_status rbd_model_destroy(rbd_model* model);
rbd_status rbd_model_dims(const rbd_model* model, int* nq, int* nv, int* n_bodies);
/* Name of the topology serving this model (static string): a compiled
 * topology's name, or "jit_<n>[f]_<hash>" for one compiled at run time. */
const char* rbd_model_topology(const rbd_model* model);

/* Compile kernels of a topology (n_bodies in 1..64, parent[i] < i
 * depth-first, floating != 0 for a free body 0) into the code-object cache
 * directory cache_dir (created if missing; NULL = the default write directory
 * described at rbd_model_create): kernel = -1 compiles all RBD_N_KERNELS of
 * them, kernel in [0, RBD_N_KERNELS) that one only, RBD_N_KERNELS + 2 f the
 * differential-IK and RBD_N_KERNELS + 2 f + 1 the operational-space-control
 * kernel of frame f (0 <= f < n_bodies; separate processes can
 * compile a topology's kernels in parallel: hiprtc compiles one program at a
 * time per process). Kernels already in the directory are kept. Needs no GPU.
 * Synchronous. Used to install a robot's kernels before its first use.
 * Errors: RBD_E_INVAL, RBD_E_COMPILE. */
#define RBD_N_KERNELS 40
rbd_status rbd_precompile_topology(int32_t n_bodies, const int32_t* parent, int floating, const char* cache_dir,
                                   int32_t kernel);

/* Forward kinematics (Sec. II): T[(i*12 + e) * ld + b] holds the world pose
 * of body i as a 3x4 row-major [R | p] (e = 4*row + col). q: [nq][ld]. */
rbd_status rbd_fk(const rbd_model* model, int64_t batch, int64_t ld, const float* q, float* T,
                  hipStream_t stream);

/* Geometric Jacobians (Sec. IV): for each of the n_frames body ids in
 * `frames` (host array, 1..256 entries, repeats allowed), the 6 x nv matrix
 * mapping qd to the world-aligned twist [v; w] of that body frame at its
 * origin. J[((f*6 + r) * nv + c) * ld + b]; columns of non-ancestor joints
 * are zero. */
rbd_status rbd_jacobian(const rbd_model* model, int64_t batch, int64_t ld, const float* q, int32_t n_frames,
                        const int32_t* frames, float* J, hipStream_t stream);

/* External forces (Eq. (1)'s J^T f term; the F_ext input of Alg. 1). f_ext,
 * where an entry point takes it, is NULL (no external forces) or a device
 * array [n_bodies * 6][ld]: element ((i*6 + c) * ld + b) is the spatial force
 * the environment applies to body i, in world axes, c = 0..2 the force and
 * c = 3..5 the moment about the world origin. It enters the joint torques as
 * -sum_i J_i^T F_i (J_i the body's Jacobian in the same world frame), so a
 * force holding a body up lowers the torque its joints need. */

/* Inverse dynamics, Eq. (1), by the recursive Newton-Euler algorithm (the
 * recursive form of Alg. 1): tau = M(q) qdd + c(q, qd) + g(q) - sum_i J_i^T
 * F_i. qdd == NULL computes the bias force h(q, qd) (with the external-force
 * term when f_ext is given). q: [nq][ld]; qd, qdd, tau: [nv][ld]. */
rbd_status rbd_rnea(const rbd_model* model, int64_t batch, int64_t ld, const float* q, const float* qd,
                    const float* qdd, const float* f_ext, float* tau, hipStream_t stream);

/* Joint-space mass matrix by the composite-rigid-body algorithm (the
 * recursive form of Alg. 2), dense and symmetric: M[(r*nv + c) * ld + b]. */
rbd_status rbd_crba(const rbd_model* model, int64_t batch, int64_t ld, const float* q, float* M,
                    hipStream_t stream);

/* Forward dynamics, Eq. (2): qdd = M(q)^-1 (tau - h(q, qd) + sum_i J_i^T F_i),
 * f_ext as above (NULL: none). One fused kernel: bias force, mass matrix and
 * its branch-sparse L^T L factorisation never leave the lane. q: [nq][ld];
 * qd, tau, qdd: [nv][ld]. */
rbd_status rbd_fwd_dyn(const rbd_model* model, int64_t batch, int64_t ld, const float* q, const float* qd,
                       const float* tau, const float* f_ext, float* qdd, hipStream_t stream);

/* Forward dynamics, Eq. (2), by the articulated-body algorithm: the same qdd
 * as rbd_fwd_dyn (up to rounding), computed in three O(n) sweeps over the
 * tree (velocities; articulated inertias and bias forces, leaves to root;
 * accelerations) without forming M. Same arguments and layout as rbd_fwd_dyn.
 * A non-positive articulated pivot yields NaN in that instance. */
rbd_status rbd_aba(const rbd_model* model, int64_t batch, int64_t ld, const float* q, const float* qd,
                   const float* tau, const float* f_ext, float* qdd, hipStream_t stream);

/* Jacobian-vector product of rbd_fwd_dyn (forward-mode AD, Sec. IV-A and
 * Fig. 2): for tangents dq [nq][ld] (raw quaternion components included),
 * dqd and dtau [nv][ld], and external-force tangents df_ext [n_bodies*6][ld]
 * (nullable: zero), dqdd = dqdd/dq dq + dqdd/dqd dqd + M^-1 dtau + M^-1
 * sum_i J_i^T dF_i [nv][ld], at the forward dynamics with external forces
 * f_ext (nullable: none; layout as for rbd_rnea). Computed as
 * M^-1 (dtau - dID/dq dq - dID/dqd dqd) at qdd = FD(q, qd, tau, F), with ID
 * including -sum_i J_i(q)^T F_i: the fused forward dynamics, a sweep of
 * tangent inverse dynamics, then a solve with M, all in one kernel (for a
 * tree of more than 16 DoFs at a batch of at most 32768, on two waves per 64
 * instances: one runs the first two sweeps while the other factors M, and
 * the right-hand side passes between them through LDS). With forces, a free
 * base's position tangent moves them relative to the robot. qdd (nullable)
 * also receives the forward dynamics. The forward dynamics may be kept in qdd
 * (or in dqdd) between the sweeps, so qdd and dqdd must not overlap
 * (RBD_E_INVAL). */
rbd_status rbd_fwd_dyn_jvp(const rbd_model* model, int64_t batch, int64_t ld, const float* q, const float* qd,
                           const float* tau, const float* f_ext, const float* dq, const float* dqd,
                           const float* dtau, const float* df_ext, float* qdd, float* dqdd, hipStream_t stream);

/* Jacobian-vector product of rbd_rnea (forward-mode AD of Eq. (1)): for
 * tangents dq [nq][ld] (raw quaternion components included), dqd and dqdd
 * [nv][ld], and external-force tangents df_ext [n_bodies*6][ld] (nullable:
 * zero), dtau = dID/dq dq + dID/dqd dqd + M dqdd - sum_i (J_i^T F_i)' [nv][ld]
 * at (q, qd, qdd) with external forces f_ext (nullable: none; layout as for
 * rbd_rnea). One sweep of tangent inverse dynamics; dtau must not overlap an
 * input (RBD_E_INVAL). */
rbd_status rbd_rnea_jvp(const rbd_model* model, int64_t batch, int64_t ld, const float* q, const float* qd,
                        const float* qdd, const float* f_ext, const float* dq, const float* dqd, const float* dqdd,
                        const float* df_ext, float* dtau, hipStream_t stream);

/* Vector-Jacobian product of rbd_rnea (reverse-mode AD of Eq. (1)) for the
 * cotangent lam [nv][ld], at (q, qd, qdd) with external forces f_ext
 * (nullable: none; layout as for rbd_rnea): g_q = lam^T dID/dq [nq][ld] (raw
 * quaternion components included), g_qd = lam^T dID/dqd [nv][ld], g_qdd =
 * lam^T dID/dqdd = M lam [nv][ld], and g_f_ext = lam^T dID/dF = -J_i lam
 * [n_bodies*6][ld] (layout of f_ext: [v_O; w] of body i's twist under joint
 * rates lam, in world axes at the world origin, negated). Every output is
 * nullable (not computed); with none the call does nothing. One sweep of the
 * adjoint of inverse dynamics. Outputs must not overlap an input or each
 * other (RBD_E_INVAL). */
rbd_status rbd_rnea_vjp(const rbd_model* model, int64_t batch, int64_t ld, const float* q, const float* qd,
                        const float* qdd, const float* f_ext, const float* lam, float* g_q, float* g_qd, float* g_qdd,
                        float* g_f_ext, hipStream_t stream);

/* Vector-Jacobian product of rbd_fwd_dyn with external forces f_ext
 * (nullable: none; layout as for rbd_rnea), for the cotangent g_qdd [nv][ld]:
 * g_q = g_qdd^T dqdd/dq [nq][ld] (raw quaternion components included; with
 * forces, a free base's position has a gradient too), g_qd = g_qdd^T
 * dqdd/dqd [nv][ld], g_tau = M^-1 g_qdd [nv][ld], and g_f_ext = g_qdd^T
 * dqdd/dF [n_bodies*6][ld]: for body i, J_i lam with lam = M^-1 g_qdd, the
 * twist of body i in world axes at the world origin, [v_O; w] (it pairs with
 * F_i = [f; n_O]). Any of the four outputs may be NULL (not computed). One
 * kernel: a solve for the forward dynamics and M^-1 g_qdd with one factor,
 * then an adjoint sweep of inverse dynamics; between the two the solutions
 * are kept in LDS (trees of more than 16 DoFs) or in the requested g_qd and
 * g_tau outputs, so the outputs must not overlap one another (RBD_E_INVAL).
 * For a tree of more than 16 DoFs at a batch of at most 32768 the two solves
 * run on two waves per 64 instances, each with its own factor, and meet in
 * LDS before the adjoint sweep (the environment variable RBD_VJP_SPLIT=0
 * turns this off, for measurement). */
rbd_status rbd_fwd_dyn_vjp(const rbd_model* model, int64_t batch, int64_t ld, const float* q, const float* qd,
                           const float* tau, const float* f_ext, const float* g_qdd, float* g_q, float* g_qd,
                           float* g_tau, float* g_f_ext, hipStream_t stream);

/* Controller workloads (Sec. IV, Sec. V and Table II: differential IK and
 * operational-space control), the plain textbook forms for one frame, fused
 * into one kernel each. frame is any body id: the last body (n_bodies - 1)
 * has kernels with the topology's others; for any other frame the kernel is
 * compiled for that frame at run time on its first use (cached on disk like
 * a new topology's kernels; RBD_E_COMPILE if that fails). target: [12][ld], the desired pose
 * [R* | p*] of the frame per instance in the layout of rbd_fk's output (R* in
 * the body's user axes). With the frame's pose (R_e, p_e) and its Jacobian J
 * as in rbd_jacobian:
 *   err = [p* - p_e; 1/2 sum_k R_e[:, k] x R*[:, k]]                (world axes)
 * rbd_diff_ik: damped least squares, qd = J^T (J J^T + damping^2 I)^-1 (gain err),
 *   qd: [nv][ld] (zero for joints off the frame's path). damping >= 0.
 * rbd_osc: a* = kp err - kd J qd, Lambda = (J M^-1 J^T)^-1, tau_null = -k_null qd,
 *   tau = J^T Lambda (a* - J M^-1 tau_null) + tau_null + h(q, qd), tau: [nv][ld]
 *   (the Jdot qd term is omitted, so forward dynamics under tau gives J qdd = a*).
 *   One sweep forms h, M = L^T L and L^-T [J^T, tau_null]; no back substitution. */
rbd_status rbd_diff_ik(const rbd_model* model, int64_t batch, int64_t ld, const float* q, int32_t frame,
                       const float* target, float gain, float damping, float* qd, hipStream_t stream);
rbd_status rbd_osc(const rbd_model* model, int64_t batch, int64_t ld, const float* q, const float* qd,
                   int32_t frame, const float* target, float kp, float kd, float k_null, float* tau,
                   hipStream_t stream);

/* Diagnostic (not on the hot path): measured FP32 FMA rate in TFLOP/s of a
 * kernel issuing ilp (1, 4 or 16) independent FMA chains per lane, launched as
 * `blocks` blocks of 256 threads with no memory traffic. At 256 blocks (one
 * wave per SIMD, the launch shape of the 35-DoF forward dynamics at batch
 * 65536) it gives the issue ceiling that shape can reach; the published FP32
 * peak assumes packed FP32, which this library does not use. Synchronous;
 * allocates and frees a small buffer. */
rbd_status rbd_diag_fma_rate(int device, int blocks, int ilp, double* tflops);

/* Diagnostic (not on the hot path): measured streaming HBM bandwidth in GB/s.
 * mode 0 writes `bytes` bytes with non-temporal 16-byte stores (the way the
 * pose, mass-matrix and Jacobian outputs are written), mode 2 with plain
 * stores; mode 1 copies `bytes` bytes (GB/s counts read + written bytes).
 * blocks = 0: one block of 256 threads per 64 KiB, each thread 16 elements
 * a block apart; blocks > 0: a grid-stride loop over that many blocks. The
 * best of 10 timed launches after 3 warm-up launches. bytes in [1 MiB,
 * 16 GiB], blocks in [0, 2^20]. Synchronous; allocates and frees its buffers
 * (device memory of bytes, twice for a copy). It is the achievable ceiling
 * the memory-bound kernels are compared with, beside the published 8 TB/s. */
rbd_status rbd_diag_hbm_rate(int device, int64_t bytes, int mode, int blocks, double* gbs);

const char* rbd_status_str(rbd_status s);
const char* rbd_last_error(void); /* message of this thread's last failed call */
int rbd_device_count(void);       /* number of visible GPUs (0 without one)    */

/* ------------------------------------------------------------------ serving
 * Continuous batching of dynamics requests: requests of mixed robots and
 * batch sizes are admitted as device memory frees up, packed into one
 * persistent launch per operation and robot (at most 16 MiB of staged data per
 * launch), replayed as a captured HIP graph, and overlapped on several
 * streams. Per-request latency is the time the batching amortises (the paper
 * finds GPU overhead dominant below about 64 instances, Sec. III-B).
 *
 * A request names a model, an operation and a batch size, and points at host
 * buffers, instance-major FP32 ([batch][n], rows of one instance contiguous):
 *   RBD_OP_FWD_DYN:     in = {q, qd, tau},          out = {qdd}
 *   RBD_OP_RNEA:        in = {q, qd, qdd},          out = {tau}
 *   RBD_OP_FWD_DYN_VJP: in = {q, qd, tau, g_qdd},   out = {g_q, g_qd, g_tau}
 * The buffers, and the model, must stay valid until rbd_server_wait reports
 * completion. The server copies inputs into its device arena, runs the batch
 * and copies the results back. A launch group that fails (a failed copy or
 * launch, a device error) fails its own requests only (RBD_E_LAUNCH); the
 * other groups and later requests are unaffected. */
typedef enum { RBD_OP_FWD_DYN = 0, RBD_OP_RNEA = 1, RBD_OP_FWD_DYN_VJP = 2 } rbd_op;

typedef struct rbd_server rbd_server;

typedef enum {
  RBD_EXEC_DEVICE = 0, /* the GPU: copies, packed kernels, completion callbacks     */
  RBD_EXEC_HOST = 1    /* no GPU: the same scheduler over host memory, for testing
                          admission, packing, completion and failure handling; a
                          group's "launch" writes, for output a of every instance i,
                          out_a[i][c] = in_(a mod n_in)[i][c mod rows] + 1000 a
                          (rows of that input); models must be host-only          */
} rbd_executor;

typedef struct {
  int device;            /* GPU id (ignored by the host executor)                   */
  size_t arena_bytes;    /* device memory for staged requests (admission budget)    */
  int n_streams;         /* concurrent launch streams, 1..8                         */
  int max_batch_requests;/* most requests packed into one launch (1..4096)          */
  double max_wait_us;    /* how long a launch may wait to gather more requests      */
  int use_graphs;        /* 1: replay captured HIP graphs, 0: plain launches        */
  int per_request;       /* 1: one launch per request (baseline mode, no packing)   */
  int executor;          /* rbd_executor                                            */
  int64_t fail_group;    /* testing: the fail_group-th launch group (counted from 1)
                            fails before anything of it is launched, as a failed
                            launch would; 0 = never                                */
  size_t max_group_bytes;/* a launch group stops growing at this many bytes of
                            staged inputs and outputs (a larger single request
                            still forms a group of its own); 0 = 16 MiB           */
} rbd_server_config;

rbd_status rbd_server_create(const rbd_server_config* cfg, rbd_server** out);
/* Queue one request; returns a ticket immediately. RBD_E_INVAL if it can never
 * fit the arena or names a bad op, size or pointer. */
rbd_status rbd_server_submit(rbd_server* s, const rbd_model* model, int op, int64_t batch,
                             const float* const* host_in, float* const* host_out, uint64_t* ticket);
/* Wait until the request finishes (timeout_s < 0: forever). On RBD_OK,
 * *req_status holds the request's own result. A ticket can be waited once. */
rbd_status rbd_server_wait(rbd_server* s, uint64_t ticket, double timeout_s, rbd_status* req_status);
/* Cancel a request that is still queued: it completes at once with status
 * RBD_E_CANCELLED (rbd_server_wait reports it; its outputs are not written).
 * RBD_E_INVAL if the ticket is unknown or its request already left the queue
 * (it then completes normally). */
rbd_status rbd_server_cancel(rbd_server* s, uint64_t ticket);
/* Latency (submit -> results in host memory) and throughput counters since
 * the last reset, and the device timeline of the launch groups finished since
 * then, from timing events each group records on its stream (before and after
 * its input copy, after its packed launch, after its copy-back). */
typedef struct {
  uint64_t requests, instances, launches;
  double p50_us, p99_us, max_us, mean_us;
  double busy_s;               /* wall time with at least one launch group in flight    */
  uint64_t groups_timed;       /* groups on the device timeline (device executor only)  */
  double gpu_kernel_s;         /* time with at least one packed launch running          */
  double gpu_kernel_overlap_s; /* time with two or more running (on different streams)  */
  double gpu_kernel_sum_s;     /* sum of the packed launches' durations                 */
  double gpu_copy_s;           /* time with at least one input or result copy running   */
  double gpu_active_s;         /* time with any copy or launch of a group running       */
} rbd_server_stats;
rbd_status rbd_server_get_stats(rbd_server* s, rbd_server_stats* out);
/* Clears the counters and starts a new device timeline (synchronises with
 * the GPU for a moment to record its origin). */
rbd_status rbd_server_reset_stats(rbd_server* s);
/* Drain outstanding requests, then free everything. */
rbd_status rbd_server_destroy(rbd_server* s);

/* Diagnostic (a measurement client, not on the hot path): an open-loop load
 * generator for a server, so that its capacity and latency are measured
 * without the overhead of a scripting-language client. Request j
 * (0 <= j < n_requests) is spec[j mod n_spec], submitted from the calling
 * thread; arrivals are Poisson at rate_per_s (exponential gaps drawn from
 * SplitMix64 seeded with `seed`), or as fast as the window allows when
 * rate_per_s is 0 (closed loop). At most `window` requests (rounded up to a
 * multiple of n_spec) are outstanding; their outputs go to buffers the
 * generator allocates and frees (host memory). One extra thread waits for
 * the tickets in order. Blocks until every request completed; *wall_s is the
 * time from the first submit to the last completion and *failed counts
 * requests whose own status was not RBD_OK. The spec's input buffers must
 * stay valid during the call. Read the server's latency figures with
 * rbd_server_get_stats (reset them before). */
typedef struct {
  const rbd_model* model;
  int op;               /* rbd_op                                 */
  int64_t batch;
  const float* in[4];   /* host inputs as for rbd_server_submit   */
} rbd_load_request;
rbd_status rbd_diag_serve_load(rbd_server* s, int n_spec, const rbd_load_request* spec, int64_t n_requests,
                               double rate_per_s, int window, uint64_t seed, double* wall_s, int64_t* failed);

/* ------------------------------------------------------------------ no allocation
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the packed
 * launch of the serving runtime over requests whose arrays are already in
 * device memory, instance-major FP32 ([batch][n]) with the inputs and outputs
 * of rbd_server_submit for `op` (unused in/out slots are ignored). The
 * descriptor table that the server keeps in memory it allocates is written,
 * by a kernel on `stream`, into a static array of 196 624 bytes that each GPU
 * holds until the process ends; the call allocates nothing and copies nothing
 * from the host. Limits per call: 1024 requests and 32768 tiles of 64
 * instances (sum over requests of ceil(batch / 64)), else RBD_E_INVAL. A
 * model whose kernels are compiled at run time must have run `op` once
 * through rbd_server_submit first (loading its code allocates), else
 * RBD_E_INVAL. Asynchronous on `stream`; the table is rewritten by every call,
 * so calls that overlap on one GPU (on different streams, or from several
 * threads) race: serialise them. Results equal those of rbd_server_submit.
 * Pointers are not dereferenced on the host and overlaps are not checked: an
 * output must not overlap an input or another request's output. */
typedef struct {
  const float* in[4];  /* device inputs, as for rbd_server_submit  */
  float* out[3];       /* device outputs, as for rbd_server_submit */
  int64_t batch;
} rbd_packed_request;
rbd_status rbd_packed_static(const rbd_model* model, int op, int n_req, const rbd_packed_request* reqs,
                             hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* RBD_H */
