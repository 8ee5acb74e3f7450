// Per-lane rigid-body algorithms for gfx950: one robot instance per lane.
//
// Everything a lane holds lives in registers: the tree is a compile-time
// type, every body loop is unrolled by template recursion, so the per-body
// transforms, velocities, forces, composite inertias and the mass-matrix factor
// are named registers and never indexed memory. Model constants are read from
// a small read-only table with uniform addresses (scalar loads, SGPR operands).
//
// Frames. Each revolute body is computed in a joint-aligned copy of its frame
// whose z axis is the joint axis, so the motion subspace is S = [e_z; 0], the
// joint rotation is Rz(q), and S^T f is just f.n.z. The constant part of the
// parent-to-child rotation, K = C_parent^T R_fix C_child, is precomputed on the
// host; R(q) = K Rz(q) costs 12 multiply-adds. Body-fixed frames keep spatial
// quantities near the bodies they describe, which matters in FP32: the root
// frame form of Alg. 1 and Alg. 2 subtracts large m|p|^2 terms for distal
// bodies.
//
// Spatial vectors are [angular; linear] (motion [w; v], force [n; f]).
// Algorithms follow the paper's problem statement (Eq. (1), Eq. (2)) in their
// recursive O(n) form, the one Alg. 1 and Alg. 2 vectorise with the ancestor
// mask U: on a GPU the parallelism is across instances, so the per-instance
// work should be the smallest, not the most parallel.
#pragma once

#include <stdint.h>

#include <type_traits>
#include <utility>

#include "rbd_shared.hpp"

#ifndef RBD_DI
#define RBD_DI __device__ __forceinline__
#endif

namespace rbd {

// =================================================================== topology
// A kinematic tree as a type: FREE says body 0 is a floating base, P... are
// the parents (depth-first order, parent[i] < i, -1 = world).
template <bool FREE, int... P>
struct Tree {
  static constexpr int N = sizeof...(P);
  static constexpr bool kFree = FREE;
  static constexpr int NV = N + (FREE ? 5 : 0);
  static constexpr int NQ = N + (FREE ? 6 : 0);
  struct Arr {
    int v[sizeof...(P)];
  };
  static constexpr Arr par_ = {{P...}};

  static constexpr int parent(int i) { return par_.v[i]; }
  static constexpr bool free_body(int i) { return FREE && i == 0; }
  static constexpr int nvb(int i) { return free_body(i) ? 6 : 1; }
  static constexpr int vofs(int i) { return (FREE && i > 0) ? i + 5 : i; }
  static constexpr int qofs(int i) { return (FREE && i > 0) ? i + 6 : i; }
  // j is i or an ancestor of i
  static constexpr bool is_anc(int j, int i) {
    for (int k = i; k >= 0; k = parent(k))
      if (k == j) return true;
    return false;
  }
  // last body of the subtree rooted at i (depth-first numbering)
  static constexpr int last(int i) {
    int m = i;
    for (int k = i + 1; k < N; ++k)
      if (is_anc(i, k)) m = k;
    return m;
  }
  static constexpr bool depth_first() {
    for (int i = 0; i < N; ++i) {
      if (parent(i) >= i || parent(i) < -1) return false;
      for (int k = i + 1; k <= last(i); ++k)
        if (!is_anc(i, k)) return false;
    }
    return true;
  }
  // ---- DoF-level tree (a free base is a chain of 6 DoFs)
  static constexpr int body_of(int k) { return FREE ? (k < 6 ? 0 : k - 5) : k; }
  static constexpr int dpar(int k) {
    if (FREE && k < 6) return k - 1;
    const int p = parent(body_of(k));
    return p < 0 ? -1 : vofs(p) + nvb(p) - 1;
  }
  static constexpr int ddepth(int k) {
    int d = 0;
    for (int j = dpar(k); j >= 0; j = dpar(j)) ++d;
    return d;
  }
  // j is a strict ancestor DoF of k
  static constexpr bool is_danc(int j, int k) {
    for (int t = dpar(k); t >= 0; t = dpar(t))
      if (t == j) return true;
    return false;
  }
  static constexpr int loff(int k) {
    int o = 0;
    for (int t = 0; t < k; ++t) o += ddepth(t);
    return o;
  }
  static constexpr int nnz() { return loff(NV); }  // off-diagonal entries of L
  // position of L[k][j] (j a strict ancestor of k) in the packed factor
  static constexpr int lidx(int k, int j) { return loff(k) + ddepth(k) - 1 - ddepth(j); }
  static_assert(N >= 1 && N <= 64, "1..64 bodies");
};

template <int I>
using ic = std::integral_constant<int, I>;
// Forces a constexpr index to be folded by the front end (an array index is not
// a constant-expression context, so a plain call would be a run-time call).
template <int V>
inline constexpr int cidx = V;

// f(ic<B>), f(ic<B+1>), ..., f(ic<E-1>). A fold over an index sequence, not a
// recursion: a recursive helper makes every level a function that holds all the
// later iterations, which is quadratic work for the optimiser.
template <int B, class F, int... Is>
RBD_DI void sfor_impl(F& f, std::integer_sequence<int, Is...>) {
  (f(ic<B + Is>{}), ...);
}
template <int B, int E, class F>
RBD_DI void sfor(F&& f) {
  if constexpr (B < E) sfor_impl<B>(f, std::make_integer_sequence<int, E - B>{});
}
// f(ic<E-1>), ..., f(ic<B>)
template <int E, class F, int... Is>
RBD_DI void sfor_rev_impl(F& f, std::integer_sequence<int, Is...>) {
  (f(ic<E - 1 - Is>{}), ...);
}
template <int B, int E, class F>
RBD_DI void sfor_rev(F&& f) {
  if constexpr (B < E) sfor_rev_impl<E>(f, std::make_integer_sequence<int, E - B>{});
}

// Runs fn(ic<J>) for J = I, parent(I), ... while the subtree of J ends at I.
template <class TP, int J, int I, class F>
RBD_DI void close_subtrees(F& fn) {
  if constexpr (J >= 0) {
    if constexpr (TP::last(J) == I) {
      fn(ic<J>{});
      close_subtrees<TP, TP::parent(J), I>(fn);
    }
  }
}

// =================================================================== algebra
struct V3 {
  float x, y, z;
};
RBD_DI V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
RBD_DI V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
RBD_DI V3 operator*(float s, V3 a) { return {s * a.x, s * a.y, s * a.z}; }
RBD_DI float dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
RBD_DI V3 cross(V3 a, V3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }

struct M3 {  // row-major
  float a[9];
};
RBD_DI V3 mul(const M3& R, V3 x) {
  return {R.a[0] * x.x + R.a[1] * x.y + R.a[2] * x.z, R.a[3] * x.x + R.a[4] * x.y + R.a[5] * x.z,
          R.a[6] * x.x + R.a[7] * x.y + R.a[8] * x.z};
}
RBD_DI V3 mulT(const M3& R, V3 x) {
  return {R.a[0] * x.x + R.a[3] * x.y + R.a[6] * x.z, R.a[1] * x.x + R.a[4] * x.y + R.a[7] * x.z,
          R.a[2] * x.x + R.a[5] * x.y + R.a[8] * x.z};
}
RBD_DI M3 mulMM(const M3& A, const M3& B) {
  M3 C;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) C.a[3 * i + j] = A.a[3 * i] * B.a[j] + A.a[3 * i + 1] * B.a[3 + j] + A.a[3 * i + 2] * B.a[6 + j];
  return C;
}
RBD_DI M3 mulMMT(const M3& A, const M3& B) {  // A B^T
  M3 C;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      C.a[3 * i + j] = A.a[3 * i] * B.a[3 * j] + A.a[3 * i + 1] * B.a[3 * j + 1] + A.a[3 * i + 2] * B.a[3 * j + 2];
  return C;
}

struct Mot {  // motion vector [w; v]
  V3 w, v;
};
struct Frc {  // force vector [n; f]
  V3 n, f;
};
RBD_DI Mot operator+(const Mot& a, const Mot& b) { return {a.w + b.w, a.v + b.v}; }
RBD_DI Frc operator+(const Frc& a, const Frc& b) { return {a.n + b.n, a.f + b.f}; }
RBD_DI Frc operator-(const Frc& a, const Frc& b) { return {a.n - b.n, a.f - b.f}; }

// Rigid-body inertia about the frame origin: mass, first moment h = m c and
// the rotational inertia about the origin (symmetric, 6 numbers).
struct Inr {
  float m;
  V3 h;
  float xx, yy, zz, xy, xz, yz;
};
RBD_DI V3 isym(const Inr& I, V3 w) {
  return {I.xx * w.x + I.xy * w.y + I.xz * w.z, I.xy * w.x + I.yy * w.y + I.yz * w.z,
          I.xz * w.x + I.yz * w.y + I.zz * w.z};
}
// I x = [Ibar w + h x v; m v - h x w]
RBD_DI Frc imul(const Inr& I, const Mot& x) { return {isym(I, x.w) + cross(I.h, x.v), I.m * x.v - cross(I.h, x.w)}; }
RBD_DI Inr operator+(const Inr& A, const Inr& B) {
  return {A.m + B.m, A.h + B.h, A.xx + B.xx, A.yy + B.yy, A.zz + B.zz, A.xy + B.xy, A.xz + B.xz, A.yz + B.yz};
}
// v x* f = [w x n + v x f; w x f]
RBD_DI Frc crf(const Mot& v, const Frc& f) { return {cross(v.w, f.n) + cross(v.v, f.f), cross(v.w, f.f)}; }
// v x m = [w x w2; w x v2 + v x w2]
RBD_DI Mot crm(const Mot& v, const Mot& m) { return {cross(v.w, m.w), cross(v.w, m.v) + cross(v.v, m.w)}; }
RBD_DI float pair(const Frc& f, const Mot& m) { return dot(f.n, m.w) + dot(f.f, m.v); }

// Fused forms: c + a x b and c + R x as chains of fused multiply-adds (the
// compiler does not reassociate a separately written sum into them).
RBD_DI V3 cross_add(V3 a, V3 b, V3 c) {
  return {__builtin_fmaf(a.y, b.z, __builtin_fmaf(-a.z, b.y, c.x)), __builtin_fmaf(a.z, b.x, __builtin_fmaf(-a.x, b.z, c.y)),
          __builtin_fmaf(a.x, b.y, __builtin_fmaf(-a.y, b.x, c.z))};
}
RBD_DI V3 mul_add(const M3& R, V3 x, V3 c) {
  return {__builtin_fmaf(R.a[0], x.x, __builtin_fmaf(R.a[1], x.y, __builtin_fmaf(R.a[2], x.z, c.x))),
          __builtin_fmaf(R.a[3], x.x, __builtin_fmaf(R.a[4], x.y, __builtin_fmaf(R.a[5], x.z, c.y))),
          __builtin_fmaf(R.a[6], x.x, __builtin_fmaf(R.a[7], x.y, __builtin_fmaf(R.a[8], x.z, c.z)))};
}

// Child frame at r (parent coords) with axes R (columns, parent coords).
// motion parent -> child: w' = R^T w, v' = R^T (v + w x r)
RBD_DI Mot xmot(const M3& R, V3 r, const Mot& m) { return {mulT(R, m.w), mulT(R, cross_add(m.w, r, m.v))}; }
// force child -> parent: f' = R f, n' = R n + r x f'
RBD_DI Frc xfrc(const M3& R, V3 r, const Frc& f) {
  const V3 fp = mul(R, f.f);
  return {mul_add(R, f.n, cross(r, fp)), fp};
}
// acc += X^T f
RBD_DI void xfrc_acc(const M3& R, V3 r, const Frc& f, Frc& acc) {
  const V3 fp = mul(R, f.f);
  acc.n = mul_add(R, f.n, cross_add(r, fp, acc.n));
  acc.f = acc.f + fp;
}
// acc += X^T I X (inertia child -> parent): h' = R h + m r,
// Ibar' = R Ibar R^T - (u r^T + r u^T - 2 (r.u) 1) - m (r r^T - |r|^2 1), u = R h
RBD_DI void xinr_acc(const M3& R, V3 r, const Inr& I, Inr& acc) {
  const V3 u = mul(R, I.h);
  // T = R * Ibar (Ibar symmetric)
  const V3 c0 = {I.xx, I.xy, I.xz}, c1 = {I.xy, I.yy, I.yz}, c2 = {I.xz, I.yz, I.zz};
  const V3 r0 = {R.a[0], R.a[1], R.a[2]}, r1 = {R.a[3], R.a[4], R.a[5]}, r2 = {R.a[6], R.a[7], R.a[8]};
  const V3 t0 = {dot(r0, c0), dot(r0, c1), dot(r0, c2)};
  const V3 t1 = {dot(r1, c0), dot(r1, c1), dot(r1, c2)};
  const V3 t2 = {dot(r2, c0), dot(r2, c1), dot(r2, c2)};
  const float ru = dot(r, u);
  const float d = __builtin_fmaf(I.m, dot(r, r), 2.0f * ru);
  const V3 mr = I.m * r;  // m r
  const V3 w = u + mr;    // u + m r, so that u r^T + r u^T + m r r^T = w r^T + r u^T on the diagonal terms below
  acc.m = acc.m + I.m;
  acc.h = acc.h + w;
  auto fdot = [](V3 a, V3 b, float c) __attribute__((always_inline)) {
    return __builtin_fmaf(a.x, b.x, __builtin_fmaf(a.y, b.y, __builtin_fmaf(a.z, b.z, c)));
  };
  acc.xx = fdot(t0, r0, __builtin_fmaf(-(u.x + w.x), r.x, acc.xx + d));
  acc.yy = fdot(t1, r1, __builtin_fmaf(-(u.y + w.y), r.y, acc.yy + d));
  acc.zz = fdot(t2, r2, __builtin_fmaf(-(u.z + w.z), r.z, acc.zz + d));
  acc.xy = fdot(t0, r1, __builtin_fmaf(-w.x, r.y, __builtin_fmaf(-r.x, u.y, acc.xy)));
  acc.xz = fdot(t0, r2, __builtin_fmaf(-w.x, r.z, __builtin_fmaf(-r.x, u.z, acc.xz)));
  acc.yz = fdot(t1, r2, __builtin_fmaf(-w.y, r.z, __builtin_fmaf(-r.y, u.z, acc.yz)));
}

// sin and cos of a joint angle of any size (continuous joints accumulate
// turns). The hardware instructions take revolutions and a bounded argument,
// and q / 2 pi in FP32 would lose the angle's absolute accuracy as |q| grows,
// so q is first reduced to r = q - k 2 pi, |r| <= pi, by Cody and Waite's
// additive reduction (Software Manual for the Elementary Functions, 1980)
// with 2 pi split into P1 + P2: P1 is 2 pi rounded to FP32, P2 the FP32
// rounding of the remainder. fma(-k, P1, q) is exact (q and k P1 are
// multiples of P1's ulp and their difference is below 8), so r carries one
// rounding, about 2^-22 absolute, for |q| up to about 10^8. For |q| <= pi,
// k = 0 and r = q exactly.
RBD_DI void fsincos(float q, float& s, float& c) {
  constexpr float kInv2Pi = 0.15915494309189535f;
  constexpr float kP1 = 6.28318548202514648f;     // 2 pi rounded to FP32
  constexpr float kP2 = -1.74845553146951715e-7f;  // 2 pi - P1, rounded to FP32
  const float k = __builtin_rintf(q * kInv2Pi);
  const float r = __builtin_fmaf(-k, kP2, __builtin_fmaf(-k, kP1, q));
  const float t = r * kInv2Pi;
  s = __builtin_amdgcn_sinf(t);
  c = __builtin_amdgcn_cosf(t);
}
RBD_DI float frsq(float x) { return __builtin_amdgcn_rsqf(x); }
RBD_DI float frcp(float x) { return __builtin_amdgcn_rcpf(x); }

// =================================================================== tables
// Per body, 32 floats: K (9, row-major), r (3), m, h (3), Ibar about the origin
// in joint-aligned axes (xx yy zz xy xz yz), C (9, row-major; joint-aligned ->
// user body axes), pad. After the bodies: gravity (3).
constexpr int kBodyStride = 32;
constexpr int kOffK = 0, kOffR = 9, kOffM = 12, kOffH = 13, kOffI = 16, kOffC = 22;

template <int I>
RBD_DI Inr load_inr(const float* __restrict__ t) {
  const float* b = t + I * kBodyStride;
  return {b[kOffM], {b[kOffH], b[kOffH + 1], b[kOffH + 2]}, b[kOffI], b[kOffI + 1], b[kOffI + 2],
          b[kOffI + 3], b[kOffI + 4], b[kOffI + 5]};
}
template <int I>
RBD_DI V3 load_r(const float* __restrict__ t) {
  const float* b = t + I * kBodyStride + kOffR;
  return {b[0], b[1], b[2]};
}
template <class TP>
RBD_DI V3 load_g(const float* __restrict__ t) {
  const float* b = t + TP::N * kBodyStride;
  return {b[0], b[1], b[2]};
}
// R = K Rz(q): columns c K0 + s K1, -s K0 + c K1, K2
template <int I>
RBD_DI M3 joint_rot_cs(const float* __restrict__ t, float c, float s) {
  const float* K = t + I * kBodyStride + kOffK;
  M3 R;
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    R.a[3 * r + 0] = c * K[3 * r] + s * K[3 * r + 1];
    R.a[3 * r + 1] = c * K[3 * r + 1] - s * K[3 * r];
    R.a[3 * r + 2] = K[3 * r + 2];
  }
  return R;
}
template <int I>
RBD_DI M3 joint_rot(const float* __restrict__ t, float q) {
  float s, c;
  fsincos(q, s, c);
  return joint_rot_cs<I>(t, c, s);
}
// Rotation of a quaternion (w,x,y,z) divided by its squared norm.
RBD_DI M3 quat_rot(float w, float x, float y, float z) {
  const float s = frcp(w * w + x * x + y * y + z * z);
  const float ww = w * w, xx = x * x, yy = y * y, zz = z * z;
  M3 R;
  R.a[0] = (ww + xx - yy - zz) * s;
  R.a[1] = 2.0f * (x * y - w * z) * s;
  R.a[2] = 2.0f * (x * z + w * y) * s;
  R.a[3] = 2.0f * (x * y + w * z) * s;
  R.a[4] = (ww - xx + yy - zz) * s;
  R.a[5] = 2.0f * (y * z - w * x) * s;
  R.a[6] = 2.0f * (x * z - w * y) * s;
  R.a[7] = 2.0f * (y * z + w * x) * s;
  R.a[8] = (ww - xx - yy + zz) * s;
  return R;
}

// Column of a composite inertia for S = [e_z; 0]: I S = [Ibar e_z; -h x e_z]
RBD_DI Frc inr_col_z(const Inr& I) { return {{I.xz, I.yz, I.zz}, {-I.h.y, I.h.x, 0.0f}}; }

// =================================================================== lane I/O
// A lane's view of a structure-of-arrays batch: element c of the lane's
// instance is row(c)[lane], with row(c) = base + c * ld the same for the whole
// wave. The row pointer lives in scalar registers and the lane offset is one
// 32-bit register shared by every access (global loads and stores take an
// SGPR base plus a 32-bit VGPR offset), so no per-access 64-bit address has
// to be kept in vector registers.
// Element `lane` of a row: the row address stays scalar and the lane's byte
// offset is a 32-bit value (batches are limited to 2^30), which is what the
// scalar-base form of global loads and stores takes; a 64-bit per-lane
// address would cost three vector instructions per access.
template <class T>
RBD_DI T* lane_ptr(T* row, uint32_t lane) {
  using B = std::conditional_t<std::is_const_v<T>, const char, char>;
  return reinterpret_cast<T*>(reinterpret_cast<B*>(row) + (lane << 2));
}
// SB selects that form; without it the compiler forms a 64-bit address per
// lane, which measured faster for small trees (more waves per SIMD hide the
// extra instructions, and their kernels are short) and slower for large ones.
template <bool SB>
struct InT {
  const float* __restrict__ base;
  int64_t ld;
  uint32_t lane;
  RBD_DI float operator()(int c) const {
    if constexpr (SB) return *lane_ptr(base + c * ld, lane);
    else return (base + c * ld)[lane];
  }
};
template <bool SB>
struct OutT {
  float* __restrict__ base;
  int64_t ld;
  uint32_t lane;
  RBD_DI void operator()(int c, float v) const {
    if constexpr (SB) *lane_ptr(base + c * ld, lane) = v;
    else (base + c * ld)[lane] = v;
  }
};
using In = InT<true>;
using Out = OutT<true>;
// The form a tree's kernels use: the scalar-base form above 16 DoFs.
template <class TP>
inline constexpr bool kScalarBase = TP::NV > 16;
// Streaming output: a non-temporal store, for the large outputs written once
// (poses, mass matrices, Jacobians) that should not displace cached data.
struct OutNT {
  float* __restrict__ base;
  int64_t ld;
  uint32_t lane;
  RBD_DI void operator()(int c, float v) const { __builtin_nontemporal_store(v, lane_ptr(base + c * ld, lane)); }
};
// A lane's own row of an instance-major array (coordinate c at p[c]). The
// row pointers come from a table in memory, so they are typed as global
// memory here: loads and stores through them are global, not flat.
using GlobalF = __attribute__((address_space(1))) float;
struct InRow {
  const GlobalF* __restrict__ p;
  RBD_DI InRow(const float* q) : p((const GlobalF*)q) {}
  RBD_DI float operator()(int c) const { return p[c]; }
};
struct OutRow {
  GlobalF* __restrict__ p;
  RBD_DI OutRow(float* q) : p((GlobalF*)q) {}
  RBD_DI void operator()(int c, float v) const { p[c] = v; }
};

// =================================================================== external forces
// Per-body external spatial forces (the F_ext input of Alg. 1), given in world
// axes as [force f; moment n about the world origin], coordinate 6 i + c of
// the lane's instance. NoFext compiles every use away.
struct NoFext {
  static constexpr bool kOn = false;
  RBD_DI float operator()(int) const { return 0.0f; }
};
struct FextIn : In {
  static constexpr bool kOn = true;
};
// Forces that may be absent as a whole (a null array reads as zero): the
// inputs of the derivative kernels, where the force cotangent or tangent is
// wanted with or without forces.
struct FextOpt : In {
  static constexpr bool kOn = true;
  RBD_DI float operator()(int c) const { return base ? In::operator()(c) : 0.0f; }
};
// The force cotangent output of the adjoint (g_F_i = J_i lam as [v_O; w], the
// twist of body i in world axes at the world origin), or none.
struct NoGF {
  static constexpr bool kOn = false;
  RBD_DI void operator()(int, float) const {}
};
struct GFOut : Out {
  static constexpr bool kOn = true;
  RBD_DI void operator()(int c, float v) const {
    if (base) Out::operator()(c, v);
  }
};

// World pose of body I's joint-aligned frame from its parent's (Rw, pw) and
// the joint rotation RI (the base rotation for a free base).
template <class TP, int I, class QI>
RBD_DI void world_pose(const float* __restrict__ t, const QI& q, const M3& RI, M3* Rw, V3* pw) {
  constexpr int P = TP::parent(I);
  if constexpr (TP::free_body(I)) {
    Rw[I] = RI;
    pw[I] = {q(0), q(1), q(2)};
  } else if constexpr (P < 0) {
    Rw[I] = RI;
    pw[I] = load_r<I>(t);
  } else {
    Rw[I] = mulMM(Rw[P], RI);
    pw[I] = mul_add(Rw[P], load_r<I>(t), pw[P]);
  }
}
// Body I's external force in its own frame: [R^T (n - p x f); R^T f].
template <int I, class FX>
RBD_DI Frc fext_body(const FX& fx, const M3& Rw, V3 pw) {
  const V3 f = {fx(6 * I), fx(6 * I + 1), fx(6 * I + 2)};
  const V3 n = {fx(6 * I + 3), fx(6 * I + 4), fx(6 * I + 5)};
  return {mulT(Rw, cross_add(f, pw, n)), mulT(Rw, f)};
}

// =================================================================== FK
// World pose of every body in the user's body axes: [R | p] row-major.
template <class TP, class QI, class TO>
RBD_DI void fk_lane(const float* __restrict__ t, const QI& q, const TO& T) {
  constexpr int N = TP::N;
  M3 Rw[N];
  V3 pw[N];
  sfor<0, N>([&](auto I_) __attribute__((always_inline)) {
    constexpr int I = decltype(I_)::value;
    constexpr int P = TP::parent(I);
    if constexpr (TP::free_body(I)) {
      Rw[I] = quat_rot(q(3), q(4), q(5), q(6));
      pw[I] = {q(0), q(1), q(2)};
    } else {
      const M3 R = joint_rot<I>(t, q(cidx<TP::qofs(I)>));
      const V3 r = load_r<I>(t);
      if constexpr (P < 0) {
        Rw[I] = R;
        pw[I] = r;
      } else {
        Rw[I] = mulMM(Rw[P], R);
        pw[I] = pw[P] + mul(Rw[P], r);
      }
    }
    // user body axes: Rw C^T
    const float* C = t + I * kBodyStride + kOffC;
    M3 Cm;
#pragma unroll
    for (int e = 0; e < 9; ++e) Cm.a[e] = C[e];
    const M3 Ro = cidx<TP::free_body(I) ? 1 : 0> ? Rw[I] : mulMMT(Rw[I], Cm);
#pragma unroll
    for (int r = 0; r < 3; ++r) {
#pragma unroll
      for (int c = 0; c < 3; ++c) T(12 * I + 4 * r + c, Ro.a[3 * r + c]);
      T(12 * I + 4 * r + 3, r == 0 ? pw[I].x : (r == 1 ? pw[I].y : pw[I].z));
    }
  });
}

// =================================================================== Jacobian
template <class TP, class QI>
RBD_DI void jac_lane(const float* __restrict__ t, const QI& q, const JacSlots& js, float* __restrict__ J, int64_t ld,
                     uint32_t lane) {
  constexpr int N = TP::N, NV = TP::NV;
  M3 Rw[N];
  V3 pw[N];
  sfor<0, N>([&](auto K_) __attribute__((always_inline)) {
    constexpr int K = decltype(K_)::value;
    constexpr int P = TP::parent(K);
    if constexpr (TP::free_body(K)) {
      Rw[K] = quat_rot(q(3), q(4), q(5), q(6));
      pw[K] = {q(0), q(1), q(2)};
    } else {
      const M3 R = joint_rot<K>(t, q(cidx<TP::qofs(K)>));
      const V3 r = load_r<K>(t);
      if constexpr (P < 0) {
        Rw[K] = R;
        pw[K] = r;
      } else {
        Rw[K] = mulMM(Rw[P], R);
        pw[K] = pw[P] + mul(Rw[P], r);
      }
    }
    const int beg = js.beg[K], end = js.beg[K + 1];
    for (int s = beg; s < end; ++s) {
      float* __restrict__ Jf = J + (int64_t)js.slot[s] * 6 * NV * ld;
      auto put = [&](int r, int c, float v) __attribute__((always_inline)) {
        __builtin_nontemporal_store(v, lane_ptr(Jf + (int64_t)(r * NV + c) * ld, lane));
      };
      sfor<0, N>([&](auto A_) __attribute__((always_inline)) {
        constexpr int A = decltype(A_)::value;
        constexpr int c0 = TP::vofs(A);
        if constexpr (TP::is_anc(A, K)) {
          const V3 d = pw[K] - pw[A];
          if constexpr (TP::free_body(A)) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              const V3 col = {Rw[A].a[c], Rw[A].a[3 + c], Rw[A].a[6 + c]};
              const V3 lin = cross(col, d);
              put(0, c0 + c, col.x); put(1, c0 + c, col.y); put(2, c0 + c, col.z);
              put(3, c0 + c, 0.0f); put(4, c0 + c, 0.0f); put(5, c0 + c, 0.0f);
              put(0, c0 + 3 + c, lin.x); put(1, c0 + 3 + c, lin.y); put(2, c0 + 3 + c, lin.z);
              put(3, c0 + 3 + c, col.x); put(4, c0 + 3 + c, col.y); put(5, c0 + 3 + c, col.z);
            }
          } else {
            const V3 z = {Rw[A].a[2], Rw[A].a[5], Rw[A].a[8]};
            const V3 lin = cross(z, d);
            put(0, c0, lin.x); put(1, c0, lin.y); put(2, c0, lin.z);
            put(3, c0, z.x); put(4, c0, z.y); put(5, c0, z.z);
          }
        } else {
#pragma unroll
          for (int c = 0; c < cidx<TP::nvb(A)>; ++c)
#pragma unroll
            for (int r = 0; r < 6; ++r) put(r, c0 + c, 0.0f);
        }
      });
    }
  });
}

// =================================================================== RNEA
// tau = ID(q, qd, qdd) - sum_i J_i^T F_ext,i; qdd may be absent (bias force),
// external forces too (NoFext). Depth-first: the backward step of a body runs
// as soon as its subtree is done, so only the current root path is live.
template <class TP, bool HAS_QDD, class QI, class QDI, class QDDI, class TO, class FX = NoFext>
RBD_DI void rnea_lane(const float* __restrict__ t, const QI& q, const QDI& qd, const QDDI& qdd, const TO& tau,
                      const FX& fx = FX{}) {
  constexpr int N = TP::N;
  constexpr int NW = FX::kOn ? N : 1;
  M3 Rw[NW];
  V3 pw[NW];
  M3 R[N];
  Mot v[N], a[N];
  Frc f[N];
  const V3 g = load_g<TP>(t);
  const V3 mg = {-g.x, -g.y, -g.z};

  auto backward = [&](auto J_) __attribute__((always_inline)) {
    constexpr int J = decltype(J_)::value;
    constexpr int P = TP::parent(J);
    if constexpr (TP::free_body(J)) {
      tau(0, f[J].f.x); tau(1, f[J].f.y); tau(2, f[J].f.z);
      tau(3, f[J].n.x); tau(4, f[J].n.y); tau(5, f[J].n.z);
    } else {
      tau(cidx<TP::vofs(J)>, f[J].n.z);
      if constexpr (P >= 0) xfrc_acc(R[J], load_r<J>(t), f[J], f[P]);
    }
  };

  sfor<0, N>([&](auto I_) __attribute__((always_inline)) {
    constexpr int I = decltype(I_)::value;
    constexpr int P = TP::parent(I);
    if constexpr (TP::free_body(I)) {
      R[I] = quat_rot(q(3), q(4), q(5), q(6));
      v[I] = {{qd(3), qd(4), qd(5)}, {qd(0), qd(1), qd(2)}};
      a[I] = {{0.0f, 0.0f, 0.0f}, mulT(R[I], mg)};
      if constexpr (HAS_QDD) a[I] = a[I] + Mot{{qdd(3), qdd(4), qdd(5)}, {qdd(0), qdd(1), qdd(2)}};
    } else {
      R[I] = joint_rot<I>(t, q(cidx<TP::qofs(I)>));
      const float w = qd(cidx<TP::vofs(I)>);
      if constexpr (P < 0) {
        v[I] = {{0.0f, 0.0f, w}, {0.0f, 0.0f, 0.0f}};
        a[I] = {{0.0f, 0.0f, 0.0f}, mulT(R[I], mg)};
      } else {
        const V3 r = load_r<I>(t);
        v[I] = xmot(R[I], r, v[P]);
        v[I].w.z = v[I].w.z + w;
        a[I] = xmot(R[I], r, a[P]);
        // + v x (S qd) = w * [wy, -wx, 0; vy, -vx, 0]
        a[I].w.x = a[I].w.x + w * v[I].w.y;
        a[I].w.y = a[I].w.y - w * v[I].w.x;
        a[I].v.x = a[I].v.x + w * v[I].v.y;
        a[I].v.y = a[I].v.y - w * v[I].v.x;
      }
      if constexpr (HAS_QDD) a[I].w.z = a[I].w.z + qdd(cidx<TP::vofs(I)>);
    }
    const Inr Ib = load_inr<I>(t);
    f[I] = imul(Ib, a[I]) + crf(v[I], imul(Ib, v[I]));
    if constexpr (FX::kOn) {
      world_pose<TP, I>(t, q, R[I], Rw, pw);
      f[I] = f[I] - fext_body<I>(fx, Rw[I], pw[I]);
    }
    // close every subtree that ends at I, deepest first
    close_subtrees<TP, I, I>(backward);
  });
}


// =================================================================== mass matrix rows
// Row of M for revolute body J: M[k][k] and M[k][j] for every ancestor DoF j
// (k = vofs(J)). F = Ic S is carried up the tree: F <- X^T F at each hop.
template <class TP, int C, class EMIT>
RBD_DI void walk_up(const float* __restrict__ t, const M3* R, Frc F, EMIT& emit) {
  constexpr int A = TP::parent(C);
  if constexpr (A >= 0) {
    F = xfrc(R[C], load_r<C>(t), F);
    emit(ic<A>{}, F);
    walk_up<TP, A>(t, R, F, emit);
  }
}

// Base block of M in [v; w] DoF order: [[m 1, [h]x^T], [[h]x, Ibar]].
RBD_DI float base_block(const Inr& I, int r, int c) {
  if (r < 3 && c < 3) return r == c ? I.m : 0.0f;
  const float hx[9] = {0.0f, -I.h.z, I.h.y, I.h.z, 0.0f, -I.h.x, -I.h.y, I.h.x, 0.0f};
  if (r >= 3 && c < 3) return hx[3 * (r - 3) + c];
  if (r < 3 && c >= 3) return hx[3 * (c - 3) + r];
  const float Ib[9] = {I.xx, I.xy, I.xz, I.xy, I.yy, I.yz, I.xz, I.yz, I.zz};
  return Ib[3 * (r - 3) + (c - 3)];
}

// =================================================================== CRBA
template <class TP, class QI>
RBD_DI void crba_lane(const float* __restrict__ t, const QI& q, float* __restrict__ Mp, int64_t ld, uint32_t lane) {
  constexpr int N = TP::N, NV = TP::NV;
  M3 R[N];
  Inr Ic[N];
  auto put = [&](int r, int c, float v) __attribute__((always_inline)) {
    __builtin_nontemporal_store(v, lane_ptr(Mp + (int64_t)(r * NV + c) * ld, lane));
  };

  auto backward = [&](auto J_) __attribute__((always_inline)) {
    constexpr int J = decltype(J_)::value;
    constexpr int P = TP::parent(J);
    if constexpr (TP::free_body(J)) {
#pragma unroll
      for (int r = 0; r < 6; ++r)
#pragma unroll
        for (int c = 0; c < 6; ++c) put(r, c, base_block(Ic[J], r, c));
    } else {
      constexpr int k = TP::vofs(J);
      put(k, k, Ic[J].zz);
      auto emit = [&](auto A_, const Frc& F) __attribute__((always_inline)) {
        constexpr int A = decltype(A_)::value;
        if constexpr (TP::free_body(A)) {
          const float e[6] = {F.f.x, F.f.y, F.f.z, F.n.x, F.n.y, F.n.z};
#pragma unroll
          for (int c = 0; c < 6; ++c) { put(k, c, e[c]); put(c, k, e[c]); }
        } else {
          put(k, cidx<TP::vofs(A)>, F.n.z);
          put(cidx<TP::vofs(A)>, k, F.n.z);
        }
      };
      walk_up<TP, J>(t, R, inr_col_z(Ic[J]), emit);
      if constexpr (P >= 0) xinr_acc(R[J], load_r<J>(t), Ic[J], Ic[P]);
    }
  };

  sfor<0, N>([&](auto I_) __attribute__((always_inline)) {
    constexpr int I = decltype(I_)::value;
    if constexpr (TP::free_body(I)) {
      R[I] = quat_rot(q(3), q(4), q(5), q(6));  // unused by M; kept for uniformity
    } else {
      R[I] = joint_rot<I>(t, q(cidx<TP::qofs(I)>));
    }
    Ic[I] = load_inr<I>(t);
    close_subtrees<TP, I, I>(backward);
  });
  // entries between DoFs of which neither is an ancestor of the other are zero
  sfor<0, NV>([&](auto K_) __attribute__((always_inline)) {
    constexpr int K = decltype(K_)::value;
    sfor<0, NV>([&](auto L_) __attribute__((always_inline)) {
      constexpr int L = decltype(L_)::value;
      if constexpr (L != K && !TP::is_danc(L, K) && !TP::is_danc(K, L)) put(K, L, 0.0f);
    });
  });
}

// =================================================================== branch-sparse L^T L
// M = L^T L with L lower triangular and, in a depth-first DoF order, nonzero
// only where M is (an entry per DoF and each of its ancestors: no fill-in).
// Rows are produced leaves to root, as subtrees close, and the first solve
// L^T y = b runs alongside for NRHS right-hand sides; a root-to-leaves sweep
// then solves L x = y.
template <class TP, int NRHS>
struct Ltl {
  static constexpr int NNZ = TP::nnz() > 0 ? TP::nnz() : 1;
  float L[NNZ];
  float Linv[TP::NV];
  float y[NRHS][TP::NV];
};

// Which right-hand-side entries can be nonzero: MASK::on(r, k) false means
// entry k of right-hand side r is structurally zero, and then so is y[r][k]
// (never stored, never read).
struct AllRhs {
  static constexpr bool on(int, int) { return true; }
};
// No right-hand side at all: the factor alone.
struct NoRhs {
  static constexpr bool on(int, int) { return false; }
};

// Row K given row K of M (Mr[j] for ancestors j, Mkk) and b_K.
template <class TP, int K, int NRHS, class MASK = AllRhs>
RBD_DI void ltl_row(Ltl<TP, NRHS>& F, const float* Mr, float Mkk, const float* bk) {
  constexpr int NV = TP::NV;
  float D = Mkk;
  sfor<K + 1, NV>([&](auto D_) __attribute__((always_inline)) {
    constexpr int Dd = decltype(D_)::value;
    if constexpr (TP::is_danc(K, Dd)) D = D - F.L[cidx<TP::lidx(Dd, K)>] * F.L[cidx<TP::lidx(Dd, K)>];
  });
  const float inv = frsq(D);
  F.Linv[K] = inv;
  sfor<0, K>([&](auto J_) __attribute__((always_inline)) {
    constexpr int Jd = decltype(J_)::value;
    if constexpr (TP::is_danc(Jd, K)) {
      float acc = Mr[Jd];
      sfor<K + 1, NV>([&](auto D_) __attribute__((always_inline)) {
        constexpr int Dd = decltype(D_)::value;
        if constexpr (TP::is_danc(K, Dd)) acc = acc - F.L[cidx<TP::lidx(Dd, K)>] * F.L[cidx<TP::lidx(Dd, Jd)>];
      });
      F.L[cidx<TP::lidx(K, Jd)>] = acc * inv;
    }
  });
  sfor<0, NRHS>([&](auto R_) __attribute__((always_inline)) {
    constexpr int r = decltype(R_)::value;
    if constexpr (MASK::on(r, K)) {
      float acc = bk[r];
      sfor<K + 1, NV>([&](auto D_) __attribute__((always_inline)) {
        constexpr int Dd = decltype(D_)::value;
        if constexpr (TP::is_danc(K, Dd) && MASK::on(r, Dd)) acc = acc - F.L[cidx<TP::lidx(Dd, K)>] * F.y[r][Dd];
      });
      F.y[r][K] = acc * inv;
    }
  });
}

// The six rows of a free base from its composite inertia; bk(r, K) gives the
// right-hand sides (base DoFs in [v; w] order).
template <class TP, int NRHS, class BK, class MASK = AllRhs>
RBD_DI void ltl_base_rows(Ltl<TP, NRHS>& F, const Inr& Ic, const BK& bk, MASK = MASK{}) {
  sfor_rev<0, 6>([&](auto K_) __attribute__((always_inline)) {
    constexpr int K = decltype(K_)::value;
    float Mr[6];
#pragma unroll
    for (int j = 0; j < K; ++j) Mr[j] = base_block(Ic, K, j);
    float b[NRHS];
#pragma unroll
    for (int r = 0; r < NRHS; ++r) b[r] = bk(r, K);
    ltl_row<TP, K, NRHS, MASK>(F, Mr, base_block(Ic, K, K), b);
  });
}

// L x = y, root to leaves; sink(r, k, x_k).
template <class TP, int NRHS, class SINK>
RBD_DI void ltl_back(const Ltl<TP, NRHS>& F, const SINK& sink) {
  constexpr int NV = TP::NV;
  sfor<0, NRHS>([&](auto R_) __attribute__((always_inline)) {
    constexpr int r = decltype(R_)::value;
    float x[NV];
    sfor<0, NV>([&](auto K_) __attribute__((always_inline)) {
      constexpr int K = decltype(K_)::value;
      float acc = F.y[r][K];
      sfor<0, K>([&](auto J_) __attribute__((always_inline)) {
        constexpr int Jd = decltype(J_)::value;
        if constexpr (TP::is_danc(Jd, K)) acc = acc - F.L[cidx<TP::lidx(K, Jd)>] * x[Jd];
      });
      x[K] = acc * F.Linv[K];
      sink(r, K, x[K]);
    });
  });
}

// y of L^T y = b for a factor computed without right-hand side (b(k) gives
// entry k): leaves first, each entry from its descendants', the same
// arithmetic as the fused sweep does while it factors.
template <class TP, class B>
RBD_DI void ltl_solve_y(Ltl<TP, 1>& F, const B& b) {
  constexpr int NV = TP::NV;
  sfor_rev<0, NV>([&](auto K_) __attribute__((always_inline)) {
    constexpr int K = decltype(K_)::value;
    float acc = b(K);
    sfor<K + 1, NV>([&](auto D_) __attribute__((always_inline)) {
      constexpr int Dd = decltype(D_)::value;
      if constexpr (TP::is_danc(K, Dd)) acc = acc - F.L[cidx<TP::lidx(Dd, K)>] * F.y[0][Dd];
    });
    F.y[0][K] = acc * F.Linv[K];
  });
}

// Row of M for revolute body J against its ancestors, into Mr (CRBA: F = Ic S
// carried up the tree).
template <class TP, int J>
RBD_DI void crba_row(const float* __restrict__ t, const M3* R, const Inr& IcJ, float* Mr) {
  auto emit = [&](auto A_, const Frc& F) __attribute__((always_inline)) {
    constexpr int A = decltype(A_)::value;
    if constexpr (TP::free_body(A)) {
      Mr[0] = F.f.x; Mr[1] = F.f.y; Mr[2] = F.f.z;
      Mr[3] = F.n.x; Mr[4] = F.n.y; Mr[5] = F.n.z;
    } else {
      Mr[cidx<TP::vofs(A)>] = F.n.z;
    }
  };
  walk_up<TP, J>(t, R, inr_col_z(IcJ), emit);
}

// =================================================================== forward dynamics
// qdd = M^-1 (tau - h) for NRHS right-hand sides (the second one, when asked,
// is an extra vector solved with the same factor); with external forces h
// includes -sum_i J_i^T F_ext,i. One depth-first sweep runs the RNEA forward
// step (bias accelerations and forces) on the way down; each closed subtree
// then does, leaves to root:
//   h_k = S^T f, f_parent += X^T f                       (RNEA backward)
//   row k of M from F = Ic S carried up, Ic_parent += X^T Ic X   (CRBA)
//   row k of the factor M = L^T L and y_k of L^T y = b   (sparse Cholesky)
// and a final root-to-leaves sweep solves L x = y.
// BIAS = false solves M x = rhs alone (no bias force, qd unused).
template <class TP, int NRHS, class QI, class QDI, class RHS, class SINK, class FX = NoFext, bool BIAS = true>
RBD_DI void fwd_dyn_lane(const float* __restrict__ t, const QI& q, const QDI& qd, const RHS& rhs, const SINK& sink,
                         const FX& fx = FX{}) {
  constexpr int N = TP::N, NV = TP::NV;
  constexpr int NW = FX::kOn ? N : 1;
  M3 Rw[NW];
  V3 pw[NW];
  M3 R[N];
  Mot v[N], a[N];
  Frc f[N];
  Inr Ic[N];
  Ltl<TP, NRHS> F;
  const V3 g = load_g<TP>(t);
  const V3 mg = {-g.x, -g.y, -g.z};

  auto backward = [&](auto J_) __attribute__((always_inline)) {
    constexpr int J = decltype(J_)::value;
    constexpr int P = TP::parent(J);
    if constexpr (TP::free_body(J)) {
      if constexpr (BIAS) {
        const float hb[6] = {f[J].f.x, f[J].f.y, f[J].f.z, f[J].n.x, f[J].n.y, f[J].n.z};
        ltl_base_rows<TP, NRHS>(F, Ic[J], [&](int r, int K) __attribute__((always_inline)) {
          return rhs(r, K) - (r == 0 ? hb[K] : 0.0f);
        });
      } else {
        ltl_base_rows<TP, NRHS>(F, Ic[J], [&](int r, int K) __attribute__((always_inline)) { return rhs(r, K); });
      }
    } else {
      constexpr int k = TP::vofs(J);
      float Mr[NV > 1 ? NV : 1];
      crba_row<TP, J>(t, R, Ic[J], Mr);
      float bk[NRHS];
#pragma unroll
      for (int r = 0; r < NRHS; ++r) bk[r] = (BIAS && r == 0) ? rhs(r, k) - f[J].n.z : rhs(r, k);
      ltl_row<TP, k, NRHS>(F, Mr, Ic[J].zz, bk);
      if constexpr (P >= 0) {
        const V3 r = load_r<J>(t);
        if constexpr (BIAS) xfrc_acc(R[J], r, f[J], f[P]);
        xinr_acc(R[J], r, Ic[J], Ic[P]);
      }
    }
  };

  sfor<0, N>([&](auto I_) __attribute__((always_inline)) {
    constexpr int I = decltype(I_)::value;
    constexpr int P = TP::parent(I);
    if constexpr (!BIAS) {
      if constexpr (TP::free_body(I)) R[I] = quat_rot(q(3), q(4), q(5), q(6));
      else R[I] = joint_rot<I>(t, q(cidx<TP::qofs(I)>));
    } else if constexpr (TP::free_body(I)) {
      R[I] = quat_rot(q(3), q(4), q(5), q(6));
      v[I] = {{qd(3), qd(4), qd(5)}, {qd(0), qd(1), qd(2)}};
      a[I] = {{0.0f, 0.0f, 0.0f}, mulT(R[I], mg)};
    } else {
      R[I] = joint_rot<I>(t, q(cidx<TP::qofs(I)>));
      const float w = qd(cidx<TP::vofs(I)>);
      if constexpr (P < 0) {
        v[I] = {{0.0f, 0.0f, w}, {0.0f, 0.0f, 0.0f}};
        a[I] = {{0.0f, 0.0f, 0.0f}, mulT(R[I], mg)};
      } else {
        const V3 r = load_r<I>(t);
        v[I] = xmot(R[I], r, v[P]);
        v[I].w.z = v[I].w.z + w;
        a[I] = xmot(R[I], r, a[P]);
        a[I].w.x = a[I].w.x + w * v[I].w.y;
        a[I].w.y = a[I].w.y - w * v[I].w.x;
        a[I].v.x = a[I].v.x + w * v[I].v.y;
        a[I].v.y = a[I].v.y - w * v[I].v.x;
      }
    }
    const Inr Ib = load_inr<I>(t);
    if constexpr (BIAS) {
      f[I] = imul(Ib, a[I]) + crf(v[I], imul(Ib, v[I]));
      if constexpr (FX::kOn) {
        world_pose<TP, I>(t, q, R[I], Rw, pw);
        f[I] = f[I] - fext_body<I>(fx, Rw[I], pw[I]);
      }
    }
    Ic[I] = Ib;
    close_subtrees<TP, I, I>(backward);
  });

  ltl_back<TP, NRHS>(F, sink);
}

// The branch-sparse L^T L factor of M(q) alone: the bias-free sweep of
// fwd_dyn_lane (joint rotations down, CRBA rows and factor rows as subtrees
// close) without right-hand sides and without the solve.
template <class TP, class QI>
RBD_DI void ltl_factor_lane(const float* __restrict__ t, const QI& q, Ltl<TP, 1>& F) {
  constexpr int N = TP::N, NV = TP::NV;
  M3 R[N];
  Inr Ic[N];
  auto backward = [&](auto J_) __attribute__((always_inline)) {
    constexpr int J = decltype(J_)::value;
    constexpr int P = TP::parent(J);
    if constexpr (TP::free_body(J)) {
      ltl_base_rows<TP, 1>(F, Ic[J], [](int, int) __attribute__((always_inline)) { return 0.0f; }, NoRhs{});
    } else {
      float Mr[NV > 1 ? NV : 1];
      crba_row<TP, J>(t, R, Ic[J], Mr);
      const float bk[1] = {0.0f};
      ltl_row<TP, TP::vofs(J), 1, NoRhs>(F, Mr, Ic[J].zz, bk);
      if constexpr (P >= 0) xinr_acc(R[J], load_r<J>(t), Ic[J], Ic[P]);
    }
  };
  sfor<0, N>([&](auto I_) __attribute__((always_inline)) {
    constexpr int I = decltype(I_)::value;
    if constexpr (TP::free_body(I)) R[I] = quat_rot(q(3), q(4), q(5), q(6));
    else R[I] = joint_rot<I>(t, q(cidx<TP::qofs(I)>));
    Ic[I] = load_inr<I>(t);
    close_subtrees<TP, I, I>(backward);
  });
}

// =================================================================== fwd_dyn tangent
// Forward-mode derivative of forward dynamics. With qdd = FD(q, qd, tau)
// known, ID(q, qd, qdd) = tau gives
//   dqdd = M^-1 (dtau - dID/dq dq - dID/dqd dqd).
// id_tangent_lane runs the tangent of inverse dynamics at (q, qd, qdd) and
// writes the right-hand side dtau - d(ID); fwd_dyn_lane without bias then
// solves with M. (One sweep doing both held the tangent state and the factor
// at once and spilled; two light sweeps are faster.)
// Tangents through a revolute joint, with dX/dq = -(S x) X:
//   dv_i = X dv_p - dq_i S x (X v_p) + S dqd_i
//   da_i = X da_p - dq_i S x (X a_p) + dv_i x S qd_i + v_i x S dqd_i
//   df_i = I da_i + dv_i x* I v_i + v_i x* I dv_i
//   df_p += X^T (df_i + dq_i S x* f_i)      (f_i the total force of body i)
//   d(ID)_i = S^T df_i.
// A free base contributes only through gravity a_0 = R^T (-g), whose
// quaternion derivative follows the normalised Hamilton rotation; its position
// does not enter body-frame dynamics.
//
// External forces F_i (fixed in the world, tangent dF_i) enter as -F_i in
// body i's force balance; in body coordinates F_i moves with the body, so
// with eta_i = X eta_parent + S dq_i the body's pose tangent (a free base
// starts from [dtheta; R^T dp], dtheta = 2 vec(conj(quat) (x) dquat) / |quat|^2),
// the body-frame force changes by -eta_i x* F_i plus dF_i in body coordinates.
// A tangent dqdd of the accelerations (DQDD with kOn) adds S dqdd_i to da_i:
// then the sweep is the full tangent of inverse dynamics.
template <class TP, class QI, class QDI, class QDDI, class DQI, class DQDI, class DTI, class OUT, class FX = NoFext,
          class DFX = NoFext, class DQDD = NoFext>
RBD_DI void id_tangent_lane(const float* __restrict__ t, const QI& q, const QDI& qd, const QDDI& qdd,
                            const DQI& dq, const DQDI& dqd, const DTI& dtau, const OUT& out, const FX& fx = FX{},
                            const DFX& dfx = DFX{}, const DQDD& dqdd = DQDD{}) {
  constexpr int N = TP::N;
  constexpr bool kExt = FX::kOn || DFX::kOn;
  constexpr int NE = kExt ? N : 1;
  M3 Rw[NE];
  V3 pw[NE];
  Mot eta[NE];
  M3 R[N];
  Mot v[N], a[N], dv[N], da[N];
  Frc f[N], df[N];
  const V3 g = load_g<TP>(t);
  const V3 mg = {-g.x, -g.y, -g.z};

  auto backward = [&](auto J_) __attribute__((always_inline)) {
    constexpr int J = decltype(J_)::value;
    constexpr int P = TP::parent(J);
    if constexpr (TP::free_body(J)) {
      const float hb[6] = {df[J].f.x, df[J].f.y, df[J].f.z, df[J].n.x, df[J].n.y, df[J].n.z};
#pragma unroll
      for (int c = 0; c < 6; ++c) out(c, dtau(c) - hb[c]);
    } else {
      constexpr int k = TP::vofs(J);
      out(k, dtau(k) - df[J].n.z);
      if constexpr (P >= 0) {
        const V3 r = load_r<J>(t);
        const float e = dq(cidx<TP::qofs(J)>);
        // df + dq S x* f: S x* [n; f] = [(-n_y, n_x, 0); (-f_y, f_x, 0)]
        Frc d = df[J];
        d.n.x = __builtin_fmaf(-e, f[J].n.y, d.n.x);
        d.n.y = __builtin_fmaf(e, f[J].n.x, d.n.y);
        d.f.x = __builtin_fmaf(-e, f[J].f.y, d.f.x);
        d.f.y = __builtin_fmaf(e, f[J].f.x, d.f.y);
        xfrc_acc(R[J], r, d, df[P]);
        xfrc_acc(R[J], r, f[J], f[P]);
      }
    }
  };

  sfor<0, N>([&](auto I_) __attribute__((always_inline)) {
    constexpr int I = decltype(I_)::value;
    constexpr int P = TP::parent(I);
    if constexpr (TP::free_body(I)) {
      const float w = q(3), x = q(4), y = q(5), z = q(6);
      const float dw = dq(3), dx = dq(4), dy = dq(5), dz = dq(6);
      R[I] = quat_rot(w, x, y, z);
      // d(R^T mg) with R = N(quat) / |quat|^2: dR = (dN - R ds) / s, ds = 2 quat . dquat
      const float s = frcp(w * w + x * x + y * y + z * z);
      const float ds = 2.0f * (w * dw + x * dx + y * dy + z * dz);
      M3 dN;
      dN.a[0] = 2.0f * (w * dw + x * dx - y * dy - z * dz);
      dN.a[1] = 2.0f * (dx * y + x * dy - dw * z - w * dz);
      dN.a[2] = 2.0f * (dx * z + x * dz + dw * y + w * dy);
      dN.a[3] = 2.0f * (dx * y + x * dy + dw * z + w * dz);
      dN.a[4] = 2.0f * (w * dw - x * dx + y * dy - z * dz);
      dN.a[5] = 2.0f * (dy * z + y * dz - dw * x - w * dx);
      dN.a[6] = 2.0f * (dx * z + x * dz - dw * y - w * dy);
      dN.a[7] = 2.0f * (dy * z + y * dz + dw * x + w * dx);
      dN.a[8] = 2.0f * (w * dw - x * dx - y * dy + z * dz);
      const V3 ag = mulT(R[I], mg);
      const V3 dag = s * (mulT(dN, mg) - ds * ag);
      v[I] = {{qd(3), qd(4), qd(5)}, {qd(0), qd(1), qd(2)}};
      a[I] = {{qdd(3), qdd(4), qdd(5)}, ag + V3{qdd(0), qdd(1), qdd(2)}};
      dv[I] = {{dqd(3), dqd(4), dqd(5)}, {dqd(0), dqd(1), dqd(2)}};
      da[I] = {{0.0f, 0.0f, 0.0f}, dag};
      if constexpr (DQDD::kOn) da[I] = da[I] + Mot{{dqdd(3), dqdd(4), dqdd(5)}, {dqdd(0), dqdd(1), dqdd(2)}};
    } else {
      R[I] = joint_rot<I>(t, q(cidx<TP::qofs(I)>));
      const float w = qd(cidx<TP::vofs(I)>);
      const float dw = dqd(cidx<TP::vofs(I)>);
      const float e = dq(cidx<TP::qofs(I)>);
      Mot ap, dap;
      if constexpr (P < 0) {
        v[I] = {{0.0f, 0.0f, w}, {0.0f, 0.0f, 0.0f}};
        dv[I] = {{0.0f, 0.0f, dw}, {0.0f, 0.0f, 0.0f}};
        ap = {{0.0f, 0.0f, 0.0f}, mulT(R[I], mg)};
        dap = {{0.0f, 0.0f, 0.0f}, {0.0f, 0.0f, 0.0f}};
      } else {
        const V3 r = load_r<I>(t);
        v[I] = xmot(R[I], r, v[P]);
        v[I].w.z = v[I].w.z + w;
        dv[I] = xmot(R[I], r, dv[P]);
        // - e S x (X v_p): the x, y parts of v_i
        dv[I].w.x = __builtin_fmaf(e, v[I].w.y, dv[I].w.x);
        dv[I].w.y = __builtin_fmaf(-e, v[I].w.x, dv[I].w.y);
        dv[I].v.x = __builtin_fmaf(e, v[I].v.y, dv[I].v.x);
        dv[I].v.y = __builtin_fmaf(-e, v[I].v.x, dv[I].v.y);
        dv[I].w.z = dv[I].w.z + dw;
        ap = xmot(R[I], r, a[P]);
        dap = xmot(R[I], r, da[P]);
      }
      // - e S x (X a_p)
      dap.w.x = __builtin_fmaf(e, ap.w.y, dap.w.x);
      dap.w.y = __builtin_fmaf(-e, ap.w.x, dap.w.y);
      dap.v.x = __builtin_fmaf(e, ap.v.y, dap.v.x);
      dap.v.y = __builtin_fmaf(-e, ap.v.x, dap.v.y);
      // v x S w and its tangent dv x S w + v x S dw
      a[I] = ap;
      a[I].w.x = __builtin_fmaf(w, v[I].w.y, a[I].w.x);
      a[I].w.y = __builtin_fmaf(-w, v[I].w.x, a[I].w.y);
      a[I].v.x = __builtin_fmaf(w, v[I].v.y, a[I].v.x);
      a[I].v.y = __builtin_fmaf(-w, v[I].v.x, a[I].v.y);
      a[I].w.z = a[I].w.z + qdd(cidx<TP::vofs(I)>);
      da[I] = dap;
      da[I].w.x = __builtin_fmaf(w, dv[I].w.y, __builtin_fmaf(dw, v[I].w.y, da[I].w.x));
      da[I].w.y = __builtin_fmaf(-w, dv[I].w.x, __builtin_fmaf(-dw, v[I].w.x, da[I].w.y));
      da[I].v.x = __builtin_fmaf(w, dv[I].v.y, __builtin_fmaf(dw, v[I].v.y, da[I].v.x));
      da[I].v.y = __builtin_fmaf(-w, dv[I].v.x, __builtin_fmaf(-dw, v[I].v.x, da[I].v.y));
      if constexpr (DQDD::kOn) da[I].w.z = da[I].w.z + dqdd(cidx<TP::vofs(I)>);
    }
    const Inr Ib = load_inr<I>(t);
    const Frc Iv = imul(Ib, v[I]);
    f[I] = imul(Ib, a[I]) + crf(v[I], Iv);
    df[I] = imul(Ib, da[I]) + crf(dv[I], Iv) + crf(v[I], imul(Ib, dv[I]));
    if constexpr (kExt) {
      world_pose<TP, I>(t, q, R[I], Rw, pw);
      if constexpr (TP::free_body(I)) {
        const float w = q(3), x = q(4), y = q(5), z = q(6);
        const float dw = dq(3), dx = dq(4), dy = dq(5), dz = dq(6);
        const float s2 = 2.0f * frcp(w * w + x * x + y * y + z * z);
        // vec(conj(quat) (x) dquat) = w du - dw u - u x du
        const V3 u = {x, y, z}, du = {dx, dy, dz};
        const V3 th = s2 * (w * du - dw * u - cross(u, du));
        eta[I] = {th, mulT(R[I], V3{dq(0), dq(1), dq(2)})};
      } else {
        constexpr int P = TP::parent(I);
        if constexpr (P < 0) eta[I] = {{0.0f, 0.0f, 0.0f}, {0.0f, 0.0f, 0.0f}};
        else eta[I] = xmot(R[I], load_r<I>(t), eta[P]);
        eta[I].w.z = eta[I].w.z + dq(cidx<TP::qofs(I)>);
      }
      const Frc fe = fext_body<I>(fx, Rw[I], pw[I]);
      const Frc dfe = fext_body<I>(dfx, Rw[I], pw[I]) - crf(eta[I], fe);
      f[I] = f[I] - fe;
      df[I] = df[I] - dfe;
    }
    close_subtrees<TP, I, I>(backward);
  });
}

// =================================================================== fwd_dyn adjoint
// Reverse-mode derivative of inverse dynamics: given (q, qd, qdd) and the
// cotangent lam of tau, accumulate dq = (dID/dq)^T lam and dqd = (dID/dqd)^T
// lam. With lam = M^-1 gbar and qdd = FD(q, qd, tau), -dq and -dqd are the
// fwd_dyn cotangents (implicit differentiation of ID(q, qd, FD) = tau).
//
// Forward (root to leaves), besides v, a, f:
//   mu_i = X_i mu_parent + S_i lam_i   (cotangent of the total force of body i)
// Backward (subtree closed), with totals f, abar = I mu + sum X^T abar_child,
//   vbar = I (mu x v) - mu x* (I v) + (S qd) x* abar + sum X^T vbar_child:
//   dq_i  = <vbar, dX/dq v_parent> + <abar, dX/dq a_parent> + <X mu_parent, S x* f>
//         with dX/dq = -(S x) X,
//   dqd_i = S^T vbar - S^T (v x* abar).
// For a free base only gravity a_0 = R^T (-g) depends on q (through the
// quaternion); its position never enters body-frame dynamics.
//
// External forces F_i (world axes, fixed in the world) add ID_ext(q) = -sum_i
// J_i^T F_i. With mu_i the twist of body i under joint rates lam (as above),
// lam^T ID_ext = -sum_i <mu_i, F_i>; its q-derivative at revolute joint k is
//   -<S_k, Wsub_k - (X mu_parent) x* Fsub_k>,  Wsub_k = sum_{i in sub(k)} mu_i x* F_i,
// Fsub_k = sum_{i in sub(k)} F_i (both carried up the tree like forces), since
// turning joint k moves every F_i of its subtree in frame k by -(S dq) x* and
// the part of mu_i below k with it. A free base moved by [dtheta; R^T dp]
// (body frame) changes every F_i by -[dtheta; R^T dp] x* F_i, so the position
// gets R Wsub_0.f and the quaternion Wsub_0.n . dtheta/dquat. (ID_0, the
// dynamics without forces, is differentiated as above with forces excluded.)
// The force cotangent g_F_i = J_i lam is mu_i in world axes at the world origin.
// With GQDD (kOn), S^T abar = M lam is written too: abar is the composite
// force of the accelerations mu (no velocity, no gravity).
template <class TP, class QI, class QDI, class QDD, class LAM, class GQ, class GQD, class FX = NoFext, class GF = NoGF,
          class GQDD = NoGF>
RBD_DI void id_adjoint_lane(const float* __restrict__ t, const QI& q, const QDI& qd, const QDD& qdd, const LAM& lam,
                            const GQ& gq, const GQD& gqd, const FX& fx = FX{}, const GF& gf = GF{},
                            const GQDD& gqdd = GQDD{}) {
  constexpr int N = TP::N;
  constexpr bool kExt = FX::kOn, kW = FX::kOn || GF::kOn;
  constexpr int NE = kExt ? N : 1, NW = kW ? N : 1;
  M3 Rw[NW];
  V3 pw[NW];
  Frc Fs[NE], Ws[NE];  // subtree sums of F_i and of mu_i x* F_i, in body coordinates
  // Only (cos q, sin q) of a body is kept between its forward and backward
  // step; R is rebuilt when needed, which keeps the live root path small.
  float cq[N], sq[N];
  M3 R0;  // base rotation (free base only)
  Mot v[N], a[N], mu[N];
  float ap[N][4];  // (X a_parent) w.x, w.y, v.x, v.y
  Frc f[N], ab[N], vb[N];
  const V3 g = load_g<TP>(t);
  const V3 mg = {-g.x, -g.y, -g.z};

  auto backward = [&](auto J_) __attribute__((always_inline)) {
    constexpr int J = decltype(J_)::value;
    constexpr int P = TP::parent(J);
    const Inr Ib = load_inr<J>(t);
    const Frc abar = imul(Ib, mu[J]) + ab[J];
    Frc vbar = imul(Ib, crm(mu[J], v[J])) - crf(mu[J], imul(Ib, v[J])) + vb[J];
    if constexpr (GQDD::kOn) {
      if constexpr (TP::free_body(J)) {
        gqdd(0, abar.f.x); gqdd(1, abar.f.y); gqdd(2, abar.f.z);
        gqdd(3, abar.n.x); gqdd(4, abar.n.y); gqdd(5, abar.n.z);
      } else {
        gqdd(cidx<TP::vofs(J)>, abar.n.z);
      }
    }
    if constexpr (TP::free_body(J)) {
      gqd(0, -vbar.f.x); gqd(1, -vbar.f.y); gqd(2, -vbar.f.z);
      gqd(3, -vbar.n.x); gqd(4, -vbar.n.y); gqd(5, -vbar.n.z);
      // d/dquat of <abar.f, R^T(-g)> = -g^T R abar, with R = N(quat) / |quat|^2
      const float w = q(3), x = q(4), y = q(5), z = q(6);
      const float s = frcp(w * w + x * x + y * y + z * z);
      const V3 u = {x, y, z}, A = abar.f;
      const float gA = dot(g, A), uA = dot(u, A), gu = dot(g, u);
      const V3 axg = cross(A, g);
      const float gRA = dot(g, mul(R0, A));  // g^T R abar
      const float dw = 2.0f * w * gA + 2.0f * dot(u, axg);
      const float dx = -2.0f * x * gA + 2.0f * g.x * uA + 2.0f * gu * A.x + 2.0f * w * axg.x;
      const float dy = -2.0f * y * gA + 2.0f * g.y * uA + 2.0f * gu * A.y + 2.0f * w * axg.y;
      const float dz = -2.0f * z * gA + 2.0f * g.z * uA + 2.0f * gu * A.z + 2.0f * w * axg.z;
      // dPhi/dquat_k = -(g^T dN/dquat_k abar - 2 quat_k g^T R abar) / |quat|^2; output -dPhi
      float g4[4] = {(dw - 2.0f * w * gRA) * s, (dx - 2.0f * x * gRA) * s, (dy - 2.0f * y * gRA) * s,
                     (dz - 2.0f * z * gRA) * s};
      V3 gp = {0.0f, 0.0f, 0.0f};
      if constexpr (kExt) {
        // position: R Wsub_0.f; quaternion: Wsub_0.n . (2 / |quat|^2) vec(conj(quat) (x) e_k)
        gp = mul(R0, Ws[J].f);
        const V3 n = Ws[J].n;
        const float s2 = 2.0f * s;
        g4[0] = __builtin_fmaf(s2, -x * n.x - y * n.y - z * n.z, g4[0]);
        g4[1] = __builtin_fmaf(s2, w * n.x - z * n.y + y * n.z, g4[1]);
        g4[2] = __builtin_fmaf(s2, z * n.x + w * n.y - x * n.z, g4[2]);
        g4[3] = __builtin_fmaf(s2, -y * n.x + x * n.y + w * n.z, g4[3]);
      }
      gq(0, gp.x); gq(1, gp.y); gq(2, gp.z);
      gq(3, g4[0]); gq(4, g4[1]); gq(5, g4[2]); gq(6, g4[3]);
    } else {
      const float w = qd(cidx<TP::vofs(J)>);
      // (S qd) x* abar = w [(-n_y, n_x, 0); (-f_y, f_x, 0)]
      vbar.n.x = vbar.n.x - w * abar.n.y;
      vbar.n.y = vbar.n.y + w * abar.n.x;
      vbar.f.x = vbar.f.x - w * abar.f.y;
      vbar.f.y = vbar.f.y + w * abar.f.x;
      // S^T (v x* abar) = z of (w x n + v x f)
      const float vxa = v[J].w.x * abar.n.y - v[J].w.y * abar.n.x + v[J].v.x * abar.f.y - v[J].v.y * abar.f.x;
      gqd(cidx<TP::vofs(J)>, -(vbar.n.z - vxa));
      // <vbar, -S x (X v_p)>: (X v_p) has the x, y parts of v
      float dq = vbar.n.x * v[J].w.y - vbar.n.y * v[J].w.x + vbar.f.x * v[J].v.y - vbar.f.y * v[J].v.x;
      dq = dq + abar.n.x * ap[J][1] - abar.n.y * ap[J][0] + abar.f.x * ap[J][3] - abar.f.y * ap[J][2];
      float dq_ext = 0.0f;
      if constexpr (kExt) {
        // <S, Wsub - (X mu_p) x* Fsub>: (X mu_p) has the x, y parts of mu
        const Frc& Fsj = Fs[J];
        dq_ext = Ws[J].n.z - (mu[J].w.x * Fsj.n.y - mu[J].w.y * Fsj.n.x + mu[J].v.x * Fsj.f.y - mu[J].v.y * Fsj.f.x);
      }
      if constexpr (P >= 0) {
        // <X mu_p, S x* f>: (X mu_p) has the x, y parts of mu
        dq = dq - mu[J].w.x * f[J].n.y + mu[J].w.y * f[J].n.x - mu[J].v.x * f[J].f.y + mu[J].v.y * f[J].f.x;
        const V3 r = load_r<J>(t);
        const M3 RJ = joint_rot_cs<J>(t, cq[J], sq[J]);
        xfrc_acc(RJ, r, f[J], f[P]);
        xfrc_acc(RJ, r, abar, ab[P]);
        xfrc_acc(RJ, r, vbar, vb[P]);
        if constexpr (kExt) {
          xfrc_acc(RJ, r, Fs[J], Fs[P]);
          xfrc_acc(RJ, r, Ws[J], Ws[P]);
        }
      }
      gq(cidx<TP::qofs(J)>, dq_ext - dq);
    }
  };

  sfor<0, N>([&](auto I_) __attribute__((always_inline)) {
    constexpr int I = decltype(I_)::value;
    constexpr int P = TP::parent(I);
    if constexpr (TP::free_body(I)) {
      R0 = quat_rot(q(3), q(4), q(5), q(6));
      v[I] = {{qd(3), qd(4), qd(5)}, {qd(0), qd(1), qd(2)}};
      a[I] = {{qdd(3), qdd(4), qdd(5)}, mulT(R0, mg) + V3{qdd(0), qdd(1), qdd(2)}};
      mu[I] = {{lam(3), lam(4), lam(5)}, {lam(0), lam(1), lam(2)}};
    } else {
      fsincos(q(cidx<TP::qofs(I)>), sq[I], cq[I]);
      const M3 RI = joint_rot_cs<I>(t, cq[I], sq[I]);
      const float w = qd(cidx<TP::vofs(I)>);
      Mot apI;
      if constexpr (P < 0) {
        v[I] = {{0.0f, 0.0f, w}, {0.0f, 0.0f, 0.0f}};
        apI = {{0.0f, 0.0f, 0.0f}, mulT(RI, mg)};
        mu[I] = {{0.0f, 0.0f, 0.0f}, {0.0f, 0.0f, 0.0f}};
      } else {
        const V3 r = load_r<I>(t);
        v[I] = xmot(RI, r, v[P]);
        v[I].w.z = v[I].w.z + w;
        apI = xmot(RI, r, a[P]);
        mu[I] = xmot(RI, r, mu[P]);
      }
      ap[I][0] = apI.w.x; ap[I][1] = apI.w.y; ap[I][2] = apI.v.x; ap[I][3] = apI.v.y;
      a[I] = apI;
      a[I].w.z = a[I].w.z + qdd(cidx<TP::vofs(I)>);
      a[I].w.x = a[I].w.x + w * v[I].w.y;
      a[I].w.y = a[I].w.y - w * v[I].w.x;
      a[I].v.x = a[I].v.x + w * v[I].v.y;
      a[I].v.y = a[I].v.y - w * v[I].v.x;
      mu[I].w.z = mu[I].w.z + lam(cidx<TP::vofs(I)>);
    }
    const Inr Ib = load_inr<I>(t);
    f[I] = imul(Ib, a[I]) + crf(v[I], imul(Ib, v[I]));
    ab[I] = Frc{{0.0f, 0.0f, 0.0f}, {0.0f, 0.0f, 0.0f}};
    vb[I] = Frc{{0.0f, 0.0f, 0.0f}, {0.0f, 0.0f, 0.0f}};
    if constexpr (kW) {
      if constexpr (TP::free_body(I)) world_pose<TP, I>(t, q, R0, Rw, pw);
      else world_pose<TP, I>(t, q, joint_rot_cs<I>(t, cq[I], sq[I]), Rw, pw);
    }
    if constexpr (kExt) {
      Fs[I] = fext_body<I>(fx, Rw[I], pw[I]);
      Ws[I] = crf(mu[I], Fs[I]);
    }
    if constexpr (GF::kOn) {
      // g_F = [v_O; w] in world axes: w = R mu.w, v_O = R mu.v + p x w
      const V3 wv = mul(Rw[I], mu[I].w);
      const V3 vo = cross_add(pw[I], wv, mul(Rw[I], mu[I].v));
      gf(6 * I, vo.x); gf(6 * I + 1, vo.y); gf(6 * I + 2, vo.z);
      gf(6 * I + 3, wv.x); gf(6 * I + 4, wv.y); gf(6 * I + 5, wv.z);
    }
    close_subtrees<TP, I, I>(backward);
  });
}

// =================================================================== ABA
// Articulated-body inertia: symmetric 6x6 [[A, B], [B^T, C]] acting on a
// motion [w; v] as n = A w + B v, f = B^T w + C v. A and C are symmetric (6
// numbers each), B is general (row-major).
struct AInr {
  float a00, a11, a22, a01, a02, a12;
  float b[9];
  float c00, c11, c22, c01, c02, c12;
};
// A rigid body: A = Ibar, B = [h]x, C = m 1.
RBD_DI AInr ainr_rigid(const Inr& I) {
  return {I.xx,  I.yy, I.zz,  I.xy, I.xz, I.yz, {0.0f, -I.h.z, I.h.y, I.h.z, 0.0f, -I.h.x, -I.h.y, I.h.x, 0.0f},
          I.m,   I.m,  I.m,   0.0f, 0.0f, 0.0f};
}
RBD_DI void ainr_add_rigid(AInr& A, const Inr& I) {
  A.a00 = A.a00 + I.xx; A.a11 = A.a11 + I.yy; A.a22 = A.a22 + I.zz;
  A.a01 = A.a01 + I.xy; A.a02 = A.a02 + I.xz; A.a12 = A.a12 + I.yz;
  A.b[1] = A.b[1] - I.h.z; A.b[2] = A.b[2] + I.h.y; A.b[3] = A.b[3] + I.h.z;
  A.b[5] = A.b[5] - I.h.x; A.b[6] = A.b[6] - I.h.y; A.b[7] = A.b[7] + I.h.x;
  A.c00 = A.c00 + I.m; A.c11 = A.c11 + I.m; A.c22 = A.c22 + I.m;
}

// Articulated inertia of a revolute body after its joint is projected out,
// Ia = IA - U U^T / D with U = IA S. For S = [e_z; 0] its angular-z row and
// column vanish, so only A's upper-left 2x2 block, the first two rows of B
// and all of C remain.
struct AInrP {
  float a00, a11, a01;
  float b[6];
  float c00, c11, c22, c01, c02, c12;
};

// acc (= or +=) X^T Ia X for the child frame at r with axes R (parent
// coordinates). X = rot(R^T) * [[1, 0], [-[r]x, 1]]: the rotation acts
// first, blockwise R M R^T, then the shift to the parent origin gives
//   A_p = A' - (B' [r]x) - (B' [r]x)^T - [r]x C' [r]x,  B_p = B' + [r]x C',
//   C_p = C'.
template <bool INIT>
RBD_DI void xainr_acc(const M3& R, V3 r, const AInrP& I, AInr& acc) {
  const float* Ra = R.a;
  // A' = P A2 P^T with P = the first two columns of R
  float wa[3][2];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    wa[i][0] = __builtin_fmaf(Ra[3 * i], I.a00, Ra[3 * i + 1] * I.a01);
    wa[i][1] = __builtin_fmaf(Ra[3 * i], I.a01, Ra[3 * i + 1] * I.a11);
  }
  float Ap[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = i; j < 3; ++j) Ap[i][j] = __builtin_fmaf(wa[i][0], Ra[3 * j], wa[i][1] * Ra[3 * j + 1]);
  // B' = (P B2) R^T, B2 = the first two rows of B
  float wb[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k) wb[i][k] = __builtin_fmaf(Ra[3 * i], I.b[k], Ra[3 * i + 1] * I.b[3 + k]);
  float Bp[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      Bp[i][j] = __builtin_fmaf(wb[i][0], Ra[3 * j], __builtin_fmaf(wb[i][1], Ra[3 * j + 1], wb[i][2] * Ra[3 * j + 2]));
  // C' = R C R^T
  const float Cm[3][3] = {{I.c00, I.c01, I.c02}, {I.c01, I.c11, I.c12}, {I.c02, I.c12, I.c22}};
  float wc[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k)
      wc[i][k] = __builtin_fmaf(Ra[3 * i], Cm[0][k], __builtin_fmaf(Ra[3 * i + 1], Cm[1][k], Ra[3 * i + 2] * Cm[2][k]));
  float Cp[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = i; j < 3; ++j)
      Cp[i][j] = __builtin_fmaf(wc[i][0], Ra[3 * j], __builtin_fmaf(wc[i][1], Ra[3 * j + 1], wc[i][2] * Ra[3 * j + 2]));
  Cp[1][0] = Cp[0][1]; Cp[2][0] = Cp[0][2]; Cp[2][1] = Cp[1][2];
  // [r]x C' (row i of [r]x times C')
  float rc[3][3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    rc[0][j] = __builtin_fmaf(r.y, Cp[2][j], -r.z * Cp[1][j]);
    rc[1][j] = __builtin_fmaf(r.z, Cp[0][j], -r.x * Cp[2][j]);
    rc[2][j] = __builtin_fmaf(r.x, Cp[1][j], -r.y * Cp[0][j]);
  }
  // T = B' [r]x and Q = ([r]x C') [r]x (symmetric), column j of [r]x:
  // (0, rz, -ry), (-rz, 0, rx), (ry, -rx, 0)
  auto times_rx = [&](const float (&M)[3][3], int i, int j) __attribute__((always_inline)) {
    return j == 0 ? __builtin_fmaf(M[i][1], r.z, -M[i][2] * r.y)
                  : (j == 1 ? __builtin_fmaf(M[i][2], r.x, -M[i][0] * r.z) : __builtin_fmaf(M[i][0], r.y, -M[i][1] * r.x));
  };
  float T[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) T[i][j] = times_rx(Bp, i, j);
  float An[6], Bn[9], Cn[6];
  const int ii[6] = {0, 1, 2, 0, 0, 1}, jj[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
  for (int e = 0; e < 6; ++e) {
    const int i = ii[e], j = jj[e];
    An[e] = Ap[i][j] - T[i][j] - T[j][i] - times_rx(rc, i, j);
    Cn[e] = Cp[i][j];
  }
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) Bn[3 * i + j] = Bp[i][j] + rc[i][j];
  if constexpr (INIT) {
    acc.a00 = An[0]; acc.a11 = An[1]; acc.a22 = An[2]; acc.a01 = An[3]; acc.a02 = An[4]; acc.a12 = An[5];
#pragma unroll
    for (int e = 0; e < 9; ++e) acc.b[e] = Bn[e];
    acc.c00 = Cn[0]; acc.c11 = Cn[1]; acc.c22 = Cn[2]; acc.c01 = Cn[3]; acc.c02 = Cn[4]; acc.c12 = Cn[5];
  } else {
    acc.a00 = acc.a00 + An[0]; acc.a11 = acc.a11 + An[1]; acc.a22 = acc.a22 + An[2];
    acc.a01 = acc.a01 + An[3]; acc.a02 = acc.a02 + An[4]; acc.a12 = acc.a12 + An[5];
#pragma unroll
    for (int e = 0; e < 9; ++e) acc.b[e] = acc.b[e] + Bn[e];
    acc.c00 = acc.c00 + Cn[0]; acc.c11 = acc.c11 + Cn[1]; acc.c22 = acc.c22 + Cn[2];
    acc.c01 = acc.c01 + Cn[3]; acc.c02 = acc.c02 + Cn[4]; acc.c12 = acc.c12 + Cn[5];
  }
}

// Solves M x = b for a symmetric positive definite n x n M, n <= 6 (unpivoted
// Cholesky; only the lower triangle of M is read).
template <int n>
RBD_DI void chol_solve(const float (&M)[6][6], const float (&b)[6], float (&x)[6]) {
  float L[6][6], inv[6], y[6];
#pragma unroll
  for (int j = 0; j < n; ++j) {
    float d = M[j][j];
#pragma unroll
    for (int k = 0; k < j; ++k) d = __builtin_fmaf(-L[j][k], L[j][k], d);
    inv[j] = frsq(d);
#pragma unroll
    for (int i = j + 1; i < n; ++i) {
      float s = M[i][j];
#pragma unroll
      for (int k = 0; k < j; ++k) s = __builtin_fmaf(-L[i][k], L[j][k], s);
      L[i][j] = s * inv[j];
    }
  }
#pragma unroll
  for (int j = 0; j < n; ++j) {
    float s = b[j];
#pragma unroll
    for (int k = 0; k < j; ++k) s = __builtin_fmaf(-L[j][k], y[k], s);
    y[j] = s * inv[j];
  }
#pragma unroll
  for (int j = n - 1; j >= 0; --j) {
    float s = y[j];
#pragma unroll
    for (int k = j + 1; k < n; ++k) s = __builtin_fmaf(-L[k][j], x[k], s);
    x[j] = s * inv[j];
  }
}
RBD_DI void chol6_solve(const float (&M)[6][6], const float (&b)[6], float (&x)[6]) { chol_solve<6>(M, b, x); }

// Solves IA x = b for a 6x6 articulated inertia, motion x from force b.
RBD_DI Mot ainr_solve(const AInr& I, const Frc& rhs) {
  const float M[6][6] = {{I.a00, I.a01, I.a02, I.b[0], I.b[1], I.b[2]},
                         {I.a01, I.a11, I.a12, I.b[3], I.b[4], I.b[5]},
                         {I.a02, I.a12, I.a22, I.b[6], I.b[7], I.b[8]},
                         {I.b[0], I.b[3], I.b[6], I.c00, I.c01, I.c02},
                         {I.b[1], I.b[4], I.b[7], I.c01, I.c11, I.c12},
                         {I.b[2], I.b[5], I.b[8], I.c02, I.c12, I.c22}};
  const float b[6] = {rhs.n.x, rhs.n.y, rhs.n.z, rhs.f.x, rhs.f.y, rhs.f.z};
  float x[6];
  chol6_solve(M, b, x);
  return {{x[0], x[1], x[2]}, {x[3], x[4], x[5]}};
}

// Forward dynamics by the articulated-body algorithm: qdd = FD(q, qd, tau),
// the O(n) alternative to forming and factoring M. One depth-first sweep does
// the velocity pass on the way down and, as each subtree closes, the
// articulated-inertia pass (leaves to root):
//   IA_i = I_i + sum X^T Ia_c X,  pA_i = v_i x* I_i v_i + sum X^T pa_c,
//   U = IA_i S, D = S^T U, u = tau_i - S^T pA_i,
//   Ia_i = IA_i - U U^T / D,  pa_i = pA_i + Ia_i c_i + U u / D,
// with c_i = v_i x S qd_i. Only U/D and u/D outlive a body's subtree; the
// acceleration pass (root to leaves) rebuilds X and v from q and qd, which is
// cheaper than holding them for every body:
//   a' = X a_parent + c_i,  qdd_i = u/D - (U/D)^T a',  a_i = a' + S qdd_i.
// Gravity is the fictitious base acceleration -g; external forces are
// subtracted from pA; a free base solves its 6x6 articulated inertia
// directly. A parent's accumulators start at its first child's contribution,
// so a chain body holds none while its subtree runs.
template <class TP, class QI, class QDI, class TI, class QDDO, class FX = NoFext>
RBD_DI void aba_lane(const float* __restrict__ t, const QI& q, const QDI& qd, const TI& tau, const QDDO& qdd,
                     const FX& fx = FX{}) {
  constexpr int N = TP::N;
  constexpr int NW = FX::kOn ? N : 1;
  M3 Rw[NW];
  V3 pw[NW];
  Frc fe[NW];  // external force in body coordinates, subtracted from pA
  float cq[N], sq[N];
  Mot v[N];
  Frc Ud[N];
  float ud[N];
  AInr acc[N];
  Frc accp[N];
  Mot a0;  // free base: total spatial acceleration (gravity included)
  const V3 g = load_g<TP>(t);
  const V3 mg = {-g.x, -g.y, -g.z};

  auto close = [&](auto J_) __attribute__((always_inline)) {
    constexpr int J = decltype(J_)::value;
    constexpr int P = TP::parent(J);
    constexpr bool kKids = TP::last(J) > J;
    const Inr Ib = load_inr<J>(t);
    Frc bias = crf(v[J], imul(Ib, v[J]));
    if constexpr (FX::kOn) bias = bias - fe[J];
    AInr IA;
    Frc pA;
    if constexpr (kKids) {
      IA = acc[J];
      ainr_add_rigid(IA, Ib);
      pA = accp[J] + bias;
    } else {
      IA = ainr_rigid(Ib);
      pA = bias;
    }
    if constexpr (TP::free_body(J)) {
      const Frc b = {{tau(3) - pA.n.x, tau(4) - pA.n.y, tau(5) - pA.n.z}, {tau(0) - pA.f.x, tau(1) - pA.f.y, tau(2) - pA.f.z}};
      a0 = ainr_solve(IA, b);
    } else {
      const Frc U = {{IA.a02, IA.a12, IA.a22}, {IA.b[6], IA.b[7], IA.b[8]}};
      const float invD = frcp(IA.a22);
      const float u = tau(cidx<TP::vofs(J)>) - pA.n.z;
      const Frc W = {invD * U.n, invD * U.f};
      Ud[J] = W;
      ud[J] = u * invD;
      if constexpr (P >= 0) {
        AInrP Ia;
        Ia.a00 = __builtin_fmaf(-U.n.x, W.n.x, IA.a00);
        Ia.a11 = __builtin_fmaf(-U.n.y, W.n.y, IA.a11);
        Ia.a01 = __builtin_fmaf(-U.n.x, W.n.y, IA.a01);
        const float uf[3] = {W.f.x, W.f.y, W.f.z};
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          Ia.b[k] = __builtin_fmaf(-U.n.x, uf[k], IA.b[k]);
          Ia.b[3 + k] = __builtin_fmaf(-U.n.y, uf[k], IA.b[3 + k]);
        }
        Ia.c00 = __builtin_fmaf(-U.f.x, W.f.x, IA.c00);
        Ia.c11 = __builtin_fmaf(-U.f.y, W.f.y, IA.c11);
        Ia.c22 = __builtin_fmaf(-U.f.z, W.f.z, IA.c22);
        Ia.c01 = __builtin_fmaf(-U.f.x, W.f.y, IA.c01);
        Ia.c02 = __builtin_fmaf(-U.f.x, W.f.z, IA.c02);
        Ia.c12 = __builtin_fmaf(-U.f.y, W.f.z, IA.c12);
        // pa = pA + Ia c + U u / D; c = w [wy, -wx, 0; vy, -vx, 0]
        const float w = qd(cidx<TP::vofs(J)>);
        const float cwx = w * v[J].w.y, cwy = -w * v[J].w.x, cvx = w * v[J].v.y, cvy = -w * v[J].v.x;
        const float ud_ = ud[J];
        Frc pa;
        pa.n.x = pA.n.x + Ia.a00 * cwx + Ia.a01 * cwy + Ia.b[0] * cvx + Ia.b[1] * cvy + U.n.x * ud_;
        pa.n.y = pA.n.y + Ia.a01 * cwx + Ia.a11 * cwy + Ia.b[3] * cvx + Ia.b[4] * cvy + U.n.y * ud_;
        pa.n.z = pA.n.z + U.n.z * ud_;
        pa.f.x = pA.f.x + Ia.b[0] * cwx + Ia.b[3] * cwy + Ia.c00 * cvx + Ia.c01 * cvy + U.f.x * ud_;
        pa.f.y = pA.f.y + Ia.b[1] * cwx + Ia.b[4] * cwy + Ia.c01 * cvx + Ia.c11 * cvy + U.f.y * ud_;
        pa.f.z = pA.f.z + Ia.b[2] * cwx + Ia.b[5] * cwy + Ia.c02 * cvx + Ia.c12 * cvy + U.f.z * ud_;
        const V3 r = load_r<J>(t);
        const M3 RJ = joint_rot_cs<J>(t, cq[J], sq[J]);
        constexpr bool kFirst = (J == P + 1);
        xainr_acc<kFirst>(RJ, r, Ia, acc[P]);
        if constexpr (kFirst) accp[P] = xfrc(RJ, r, pa);
        else xfrc_acc(RJ, r, pa, accp[P]);
      }
    }
  };

  // velocity pass (root to leaves) with the articulated pass on subtree close
  sfor<0, N>([&](auto I_) __attribute__((always_inline)) {
    constexpr int I = decltype(I_)::value;
    constexpr int P = TP::parent(I);
    if constexpr (TP::free_body(I)) {
      v[I] = {{qd(3), qd(4), qd(5)}, {qd(0), qd(1), qd(2)}};
      if constexpr (FX::kOn) world_pose<TP, I>(t, q, quat_rot(q(3), q(4), q(5), q(6)), Rw, pw);
    } else {
      fsincos(q(cidx<TP::qofs(I)>), sq[I], cq[I]);
      const float w = qd(cidx<TP::vofs(I)>);
      const M3 RI = joint_rot_cs<I>(t, cq[I], sq[I]);
      if constexpr (P < 0) {
        v[I] = {{0.0f, 0.0f, w}, {0.0f, 0.0f, 0.0f}};
      } else {
        v[I] = xmot(RI, load_r<I>(t), v[P]);
        v[I].w.z = v[I].w.z + w;
      }
      if constexpr (FX::kOn) world_pose<TP, I>(t, q, RI, Rw, pw);
    }
    if constexpr (FX::kOn) fe[I] = fext_body<I>(fx, Rw[I], pw[I]);
    close_subtrees<TP, I, I>(close);
  });

  // acceleration pass (root to leaves), velocities rebuilt on the way
  Mot a[N], vv[N];
  sfor<0, N>([&](auto I_) __attribute__((always_inline)) {
    constexpr int I = decltype(I_)::value;
    constexpr int P = TP::parent(I);
    if constexpr (TP::free_body(I)) {
      const V3 ag = mulT(quat_rot(q(3), q(4), q(5), q(6)), mg);
      a[I] = a0;
      vv[I] = {{qd(3), qd(4), qd(5)}, {qd(0), qd(1), qd(2)}};
      qdd(0, a0.v.x - ag.x); qdd(1, a0.v.y - ag.y); qdd(2, a0.v.z - ag.z);
      qdd(3, a0.w.x); qdd(4, a0.w.y); qdd(5, a0.w.z);
    } else {
      float s, c;
      fsincos(q(cidx<TP::qofs(I)>), s, c);
      const M3 RI = joint_rot_cs<I>(t, c, s);
      const float w = qd(cidx<TP::vofs(I)>);
      Mot ap;
      if constexpr (P < 0) {
        vv[I] = {{0.0f, 0.0f, w}, {0.0f, 0.0f, 0.0f}};
        ap = {{0.0f, 0.0f, 0.0f}, mulT(RI, mg)};
      } else {
        const V3 r = load_r<I>(t);
        vv[I] = xmot(RI, r, vv[P]);
        vv[I].w.z = vv[I].w.z + w;
        ap = xmot(RI, r, a[P]);
        ap.w.x = __builtin_fmaf(w, vv[I].w.y, ap.w.x);
        ap.w.y = __builtin_fmaf(-w, vv[I].w.x, ap.w.y);
        ap.v.x = __builtin_fmaf(w, vv[I].v.y, ap.v.x);
        ap.v.y = __builtin_fmaf(-w, vv[I].v.x, ap.v.y);
      }
      const float x = ud[I] - pair(Ud[I], ap);
      qdd(cidx<TP::vofs(I)>, x);
      ap.w.z = ap.w.z + x;
      a[I] = ap;
    }
  });
}

// =================================================================== controller workloads
// One end-effector frame E (a compile-time body id), a target pose [R* | p*]
// (12 numbers, row-major like the FK output) per instance. Pose error in world
// axes: err = [p* - p_E; 1/2 sum_k R_E[:, k] x R*[:, k]] with R_E the user
// axes of body E. J is E's world-aligned Jacobian at its origin (rows [v; w]);
// its column for a DoF is zero unless the DoF's body is E or an ancestor (the
// path of E).

// right-hand sides 0..5 (the rows of J) vanish off the path of E
template <class TP, int E>
struct PathRhs {
  static constexpr bool on(int r, int k) { return r >= 6 || TP::is_anc(TP::body_of(k), E); }
};

template <class TP, int E, class TGT>
RBD_DI void pose_error(const float* __restrict__ t, const M3& RwE, V3 pE, const TGT& tgt, float (&err)[6]) {
  M3 Ru = RwE;  // user axes: Rw C^T (a free base has none of its own)
  if constexpr (!TP::free_body(E)) {
    const float* C = t + E * kBodyStride + kOffC;
    M3 Cm;
#pragma unroll
    for (int e = 0; e < 9; ++e) Cm.a[e] = C[e];
    Ru = mulMMT(RwE, Cm);
  }
  V3 rot = {0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const V3 a = {Ru.a[k], Ru.a[3 + k], Ru.a[6 + k]};
    const V3 b = {tgt(k), tgt(4 + k), tgt(8 + k)};
    rot = cross_add(a, b, rot);
  }
  err[0] = tgt(3) - pE.x; err[1] = tgt(7) - pE.y; err[2] = tgt(11) - pE.z;
  err[3] = 0.5f * rot.x; err[4] = 0.5f * rot.y; err[5] = 0.5f * rot.z;
}

// Column c (0..5) of J for the DoFs of a free base with world pose (R0, p0).
RBD_DI void base_jcol(const M3& R0, V3 p0, V3 pE, int c, float (&col)[6]) {
  const V3 ax = {R0.a[c % 3], R0.a[3 + c % 3], R0.a[6 + c % 3]};
  if (c < 3) {
    col[0] = ax.x; col[1] = ax.y; col[2] = ax.z; col[3] = 0.0f; col[4] = 0.0f; col[5] = 0.0f;
  } else {
    const V3 lin = cross(ax, pE - p0);
    col[0] = lin.x; col[1] = lin.y; col[2] = lin.z; col[3] = ax.x; col[4] = ax.y; col[5] = ax.z;
  }
}
// Column of J for a revolute body K with world pose (Rw, pw): [z x (pE - p); z].
RBD_DI void rev_jcol(const M3& Rw, V3 pw, V3 pE, float (&col)[6]) {
  const V3 z = {Rw.a[2], Rw.a[5], Rw.a[8]};
  const V3 lin = cross(z, pE - pw);
  col[0] = lin.x; col[1] = lin.y; col[2] = lin.z; col[3] = z.x; col[4] = z.y; col[5] = z.z;
}

// Differential IK by damped least squares: qd = J^T (J J^T + lam^2 I)^-1 (k err).
// Only E's path is visited: world poses, Jacobian columns and a normal matrix.
// With fewer than six DoFs on the path the same qd is formed as
// (J^T J + lam^2 I)^-1 J^T (k err): there J J^T is singular, and the 6x6 form
// would build large components of w that J^T then cancels in FP32.
template <class TP, int E>
struct EPath {
  static constexpr int count() {
    int c = 0;
    for (int k = 0; k < TP::NV; ++k) c += TP::is_anc(TP::body_of(k), E) ? 1 : 0;
    return c;
  }
  static constexpr int slot(int k) {  // position of DoF k among the path's DoFs
    int c = 0;
    for (int j = 0; j < k; ++j) c += TP::is_anc(TP::body_of(j), E) ? 1 : 0;
    return c;
  }
};

template <class TP, int E, class QI, class TGT, class QDO>
RBD_DI void diff_ik_lane(const float* __restrict__ t, const QI& q, const TGT& tgt, float gain, float lam2,
                         const QDO& qdo) {
  constexpr int N = TP::N, NV = TP::NV;
  constexpr int NP = EPath<TP, E>::count();
  M3 Rw[N];
  V3 pw[N];
  sfor<0, E + 1>([&](auto I_) __attribute__((always_inline)) {
    constexpr int I = decltype(I_)::value;
    if constexpr (TP::is_anc(I, E)) {
      M3 RI;
      if constexpr (TP::free_body(I)) RI = quat_rot(q(3), q(4), q(5), q(6));
      else RI = joint_rot<I>(t, q(cidx<TP::qofs(I)>));
      world_pose<TP, I>(t, q, RI, Rw, pw);
    }
  });
  const V3 pE = pw[E];
  float err[6];
  pose_error<TP, E>(t, Rw[E], pE, tgt, err);
  float b[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) b[i] = gain * err[i];
  float Jc[NV][6];
  sfor<0, N>([&](auto I_) __attribute__((always_inline)) {
    constexpr int I = decltype(I_)::value;
    if constexpr (TP::is_anc(I, E)) {
      if constexpr (TP::free_body(I)) {
#pragma unroll
        for (int c = 0; c < 6; ++c) base_jcol(Rw[I], pw[I], pE, c, Jc[c]);
      } else {
        rev_jcol(Rw[I], pw[I], pE, Jc[cidx<TP::vofs(I)>]);
      }
    }
  });
  float A[6][6];
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = 0; j < 6; ++j) A[i][j] = (i == j) ? lam2 : 0.0f;
  if constexpr (NP >= 6) {
    // (J J^T + lam^2 I) w = k err, qd = J^T w
    sfor<0, NV>([&](auto K_) __attribute__((always_inline)) {
      constexpr int K = decltype(K_)::value;
      if constexpr (TP::is_anc(TP::body_of(K), E)) {
#pragma unroll
        for (int i = 0; i < 6; ++i)
#pragma unroll
          for (int j = 0; j <= i; ++j) A[i][j] = __builtin_fmaf(Jc[K][i], Jc[K][j], A[i][j]);
      }
    });
    float w[6];
    chol_solve<6>(A, b, w);
    sfor<0, NV>([&](auto K_) __attribute__((always_inline)) {
      constexpr int K = decltype(K_)::value;
      if constexpr (TP::is_anc(TP::body_of(K), E)) {
        float x = 0.0f;
#pragma unroll
        for (int i = 0; i < 6; ++i) x = __builtin_fmaf(Jc[K][i], w[i], x);
        qdo(K, x);
      } else {
        qdo(K, 0.0f);
      }
    });
  } else {
    // (J^T J + lam^2 I) x = J^T k err over the path's DoFs
    float rhs[6], x[6];
    sfor<0, NV>([&](auto K_) __attribute__((always_inline)) {
      constexpr int K = decltype(K_)::value;
      if constexpr (TP::is_anc(TP::body_of(K), E)) {
        constexpr int a = EPath<TP, E>::slot(K);
        float r = 0.0f;
#pragma unroll
        for (int i = 0; i < 6; ++i) r = __builtin_fmaf(Jc[K][i], b[i], r);
        rhs[a] = r;
        sfor<0, K + 1>([&](auto L_) __attribute__((always_inline)) {
          constexpr int L = decltype(L_)::value;
          if constexpr (TP::is_anc(TP::body_of(L), E)) {
            constexpr int c = EPath<TP, E>::slot(L);
#pragma unroll
            for (int i = 0; i < 6; ++i) A[a][c] = __builtin_fmaf(Jc[K][i], Jc[L][i], A[a][c]);
          }
        });
      }
    });
    chol_solve<NP>(A, rhs, x);
    sfor<0, NV>([&](auto K_) __attribute__((always_inline)) {
      constexpr int K = decltype(K_)::value;
      if constexpr (TP::is_anc(TP::body_of(K), E)) qdo(K, x[cidx<EPath<TP, E>::slot(K)>]);
      else qdo(K, 0.0f);
    });
  }
}

// Operational-space control (Khatib's form, the Jdot qd term omitted):
//   a* = kp err - kd J qd,  tau_null = -k_null qd,
//   tau = J^T Lambda (a* - J M^-1 tau_null) + tau_null + h,  Lambda^-1 = J M^-1 J^T.
// Two depth-first sweeps over the branch-sparse factor M = L^T L (as in
// fwd_dyn_lane); L is never used after its sweep, so no back substitution is
// needed. One sweep carrying all seven right-hand sides holds more than the
// register file and spills; two sweeps each hold about what forward dynamics
// holds.
//   osc_sweep_bias: bias force h and the factor with one right-hand side,
//     y = L^-T tau_null. It writes h + tau_null for every DoF and returns y on
//     E's path and a* (pose error and twist of E, in E's axes).
//   osc_sweep_task: the factor again with the six rows of J as right-hand
//     sides, Y = L^-T J^T. Lambda^-1 = Y^T Y and J M^-1 tau_null = Y^T y
//     accumulate as the path's DoFs close; a 6x6 solve gives the task wrench
//     z, and J^T z (z applied at E and carried down E's path like a body
//     force) is added to the torques the first sweep wrote.
// The task space is expressed in E's own frame: the second sweep carries one
// transform up E's path, the rotation A_J = R_{E<-J} and the origin o_J of
// body J in E's frame (A_E = I, o_E = 0; A_P = A_J R_J^T, o_P = o_J - A_P r_J),
// and J's column is [o_J x z_J; z_J] with z_J = A_J e_z.
template <class TP, int E, class QI, class QDI, class TGT, class TO>
RBD_DI void osc_sweep_bias(const float* __restrict__ t, const QI& q, const QDI& qd, const TGT& tgt, float kp,
                           float kd, float kn, const TO& tau, float (&ypath)[TP::NV], float (&astar)[6]) {
  constexpr int N = TP::N, NV = TP::NV;
  M3 R[N], Rw[N];
  V3 pw[N];
  Mot v[N], a[N];
  Frc f[N];
  Inr Ic[N];
  Ltl<TP, 1> F;
  const V3 g = load_g<TP>(t);
  const V3 mg = {-g.x, -g.y, -g.z};

  auto backward = [&](auto J_) __attribute__((always_inline)) {
    constexpr int J = decltype(J_)::value;
    constexpr int P = TP::parent(J);
    if constexpr (TP::free_body(J)) {
      ltl_base_rows<TP, 1>(F, Ic[J], [&](int, int K) __attribute__((always_inline)) { return -kn * qd(K); });
      const float hb[6] = {f[J].f.x, f[J].f.y, f[J].f.z, f[J].n.x, f[J].n.y, f[J].n.z};
      sfor<0, 6>([&](auto K_) __attribute__((always_inline)) {
        constexpr int K = decltype(K_)::value;
        ypath[K] = F.y[0][K];
        tau(K, __builtin_fmaf(-kn, qd(K), hb[K]));
      });
    } else {
      constexpr int k = TP::vofs(J);
      float Mr[NV > 1 ? NV : 1];
      crba_row<TP, J>(t, R, Ic[J], Mr);
      const float bk[1] = {-kn * qd(k)};
      ltl_row<TP, k, 1>(F, Mr, Ic[J].zz, bk);
      if constexpr (TP::is_anc(J, E)) ypath[k] = F.y[0][k];
      tau(k, f[J].n.z + bk[0]);
      if constexpr (P >= 0) {
        const V3 r = load_r<J>(t);
        xfrc_acc(R[J], r, f[J], f[P]);
        xinr_acc(R[J], r, Ic[J], Ic[P]);
      }
    }
  };

  sfor<0, N>([&](auto I_) __attribute__((always_inline)) {
    constexpr int I = decltype(I_)::value;
    constexpr int P = TP::parent(I);
    if constexpr (TP::free_body(I)) {
      R[I] = quat_rot(q(3), q(4), q(5), q(6));
      v[I] = {{qd(3), qd(4), qd(5)}, {qd(0), qd(1), qd(2)}};
      a[I] = {{0.0f, 0.0f, 0.0f}, mulT(R[I], mg)};
    } else {
      R[I] = joint_rot<I>(t, q(cidx<TP::qofs(I)>));
      const float w = qd(cidx<TP::vofs(I)>);
      if constexpr (P < 0) {
        v[I] = {{0.0f, 0.0f, w}, {0.0f, 0.0f, 0.0f}};
        a[I] = {{0.0f, 0.0f, 0.0f}, mulT(R[I], mg)};
      } else {
        const V3 r = load_r<I>(t);
        v[I] = xmot(R[I], r, v[P]);
        v[I].w.z = v[I].w.z + w;
        a[I] = xmot(R[I], r, a[P]);
        a[I].w.x = a[I].w.x + w * v[I].w.y;
        a[I].w.y = a[I].w.y - w * v[I].w.x;
        a[I].v.x = a[I].v.x + w * v[I].v.y;
        a[I].v.y = a[I].v.y - w * v[I].v.x;
      }
    }
    if constexpr (TP::is_anc(I, E)) world_pose<TP, I>(t, q, R[I], Rw, pw);
    if constexpr (I == E) {
      float err[6];
      pose_error<TP, E>(t, Rw[E], pw[E], tgt, err);
      // the world-axes error turned into E's axes; E's twist in its own axes is its body velocity
      const V3 el = mulT(Rw[E], V3{err[0], err[1], err[2]}), ea = mulT(Rw[E], V3{err[3], err[4], err[5]});
      const float e6[6] = {el.x, el.y, el.z, ea.x, ea.y, ea.z};
      const float tw[6] = {v[E].v.x, v[E].v.y, v[E].v.z, v[E].w.x, v[E].w.y, v[E].w.z};
#pragma unroll
      for (int i = 0; i < 6; ++i) astar[i] = kp * e6[i] - kd * tw[i];
    }
    const Inr Ib = load_inr<I>(t);
    f[I] = imul(Ib, a[I]) + crf(v[I], imul(Ib, v[I]));
    Ic[I] = Ib;
    close_subtrees<TP, I, I>(backward);
  });
}

// TI reads back what TO wrote in the first sweep.
template <class TP, int E, class QI, class TO, class TI>
RBD_DI void osc_sweep_task(const float* __restrict__ t, const QI& q, const float (&ypath)[TP::NV],
                           const float (&astar)[6], const TO& tau, const TI& tau_in) {
  constexpr int N = TP::N, NV = TP::NV;
  using MK = PathRhs<TP, E>;
  M3 R[N];
  Inr Ic[N];
  Ltl<TP, 6> F;
  float G[6][6], c6[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    c6[i] = 0.0f;
#pragma unroll
    for (int j = 0; j < 6; ++j) G[i][j] = 0.0f;
  }
  M3 At = {{1.0f, 0.0f, 0.0f, 0.0f, 1.0f, 0.0f, 0.0f, 0.0f, 1.0f}};  // A_J of the next path body to close
  V3 ot = {0.0f, 0.0f, 0.0f};                                         // o_J

  auto accumulate = [&](auto K_) __attribute__((always_inline)) {
    constexpr int K = decltype(K_)::value;
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      c6[i] = __builtin_fmaf(F.y[i][K], ypath[K], c6[i]);
#pragma unroll
      for (int j = 0; j <= i; ++j) G[i][j] = __builtin_fmaf(F.y[i][K], F.y[j][K], G[i][j]);
    }
  };

  auto backward = [&](auto J_) __attribute__((always_inline)) {
    constexpr int J = decltype(J_)::value;
    constexpr int P = TP::parent(J);
    constexpr bool kPath = TP::is_anc(J, E);
    if constexpr (TP::free_body(J)) {
      // E-frame columns of the base DoFs: [A e_c; 0] (linear), [o x A e_c; A e_c] (angular)
      float cols[6][6];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const V3 ax = {At.a[c], At.a[3 + c], At.a[6 + c]};
        const V3 lin = cross(ot, ax);
        cols[c][0] = ax.x; cols[c][1] = ax.y; cols[c][2] = ax.z; cols[c][3] = 0.0f; cols[c][4] = 0.0f; cols[c][5] = 0.0f;
        cols[c + 3][0] = lin.x; cols[c + 3][1] = lin.y; cols[c + 3][2] = lin.z;
        cols[c + 3][3] = ax.x; cols[c + 3][4] = ax.y; cols[c + 3][5] = ax.z;
      }
      ltl_base_rows<TP, 6>(F, Ic[J], [&](int r, int K) __attribute__((always_inline)) { return cols[K][r]; }, MK{});
      sfor<0, 6>([&](auto K_) __attribute__((always_inline)) { accumulate(K_); });
    } else {
      constexpr int k = TP::vofs(J);
      float Mr[NV > 1 ? NV : 1];
      crba_row<TP, J>(t, R, Ic[J], Mr);
      float bk[6];
      if constexpr (kPath) {
        const V3 z = {At.a[2], At.a[5], At.a[8]};
        const V3 lin = cross(ot, z);
        bk[0] = lin.x; bk[1] = lin.y; bk[2] = lin.z; bk[3] = z.x; bk[4] = z.y; bk[5] = z.z;
      }
      ltl_row<TP, k, 6, MK>(F, Mr, Ic[J].zz, bk);
      if constexpr (kPath) accumulate(ic<k>{});
      if constexpr (P >= 0) {
        const V3 r = load_r<J>(t);
        xinr_acc(R[J], r, Ic[J], Ic[P]);
        if constexpr (kPath) {
          At = mulMMT(At, R[J]);
          ot = ot - mul(At, r);
        }
      }
    }
  };

  sfor<0, N>([&](auto I_) __attribute__((always_inline)) {
    constexpr int I = decltype(I_)::value;
    if constexpr (TP::free_body(I)) R[I] = quat_rot(q(3), q(4), q(5), q(6));
    else R[I] = joint_rot<I>(t, q(cidx<TP::qofs(I)>));
    Ic[I] = load_inr<I>(t);
    close_subtrees<TP, I, I>(backward);
  });

  // task wrench z = Lambda (a* - J M^-1 tau_null)
  float rhs[6], z[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) rhs[i] = astar[i] - c6[i];
  chol6_solve(G, rhs, z);
  // J^T z: the wrench [z_lin; z_ang] at E's origin (E's axes), carried down E's path
  Frc w = {V3{z[3], z[4], z[5]}, V3{z[0], z[1], z[2]}};
  sfor_rev<0, E + 1>([&](auto K_) __attribute__((always_inline)) {
    constexpr int K = decltype(K_)::value;
    constexpr int P = TP::parent(K);
    if constexpr (TP::is_anc(K, E)) {
      if constexpr (TP::free_body(K)) {
        const float wb[6] = {w.f.x, w.f.y, w.f.z, w.n.x, w.n.y, w.n.z};
#pragma unroll
        for (int c = 0; c < 6; ++c) tau(c, tau_in(c) + wb[c]);
      } else {
        constexpr int k = TP::vofs(K);
        tau(k, tau_in(k) + w.n.z);
        if constexpr (P >= 0) w = xfrc(joint_rot<K>(t, q(cidx<TP::qofs(K)>)), load_r<K>(t), w);
      }
    }
  });
}

}  // namespace rbd
