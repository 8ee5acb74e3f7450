// FP64 CPU oracle for batched rigid-body kinematics and dynamics.
//
// TEST INFRASTRUCTURE ONLY. Only the tests, the smoke check and the CPU
// baseline leg of the benchmark load this library. It shares no code, header,
// table or constant with the GPU library, and the GPU library never calls it.
//
// What it computes (paper: Sec. II, Eq. (1) and Eq. (2); Sec. III, Alg. 1 and
// Alg. 2 define the same quantities in a vectorised form):
//   * forward kinematics 0T_i(q) of every body frame (Sec. II);
//   * the world-aligned geometric Jacobian of any body frame (Sec. IV, the
//     analytical Jacobians the library provides);
//   * inverse dynamics tau = M(q) qdd + c(q,qd) + g(q), Eq. (1), by the
//     recursive Newton-Euler algorithm in body coordinates (the recursive
//     form that the paper's Alg. 1 vectorises; Featherstone, RBDA Table 5.1);
//   * the joint-space mass matrix M(q) by the composite-rigid-body algorithm
//     (the recursive form of Alg. 2; RBDA Table 6.2);
//   * forward dynamics qdd = M^-1 (tau - c - g), Eq. (2), three independent
//     ways: dense Cholesky L L^T without pivoting, the branch-sparse L^T L
//     factorisation of RBDA Sec. 6.5, and the articulated-body algorithm
//     (RBDA Table 7.1) which never forms M (Sec. II names all three
//     Featherstone algorithms; Sec. VI-A, footnote, prefers a Cholesky solve);
//   * the vector-Jacobian product of forward dynamics by central finite
//     differences (reverse-mode derivatives, Sec. I and Sec. VI-A).
//
// Conventions. Spatial vectors inside this file are Featherstone's
// [angular; linear]. Generalised coordinates: a revolute joint has one q and
// one qd. A free joint (body 0 only) has q = [p_world(3); quat w,x,y,z (4)]
// and qd = [v_B; w_B], the body-frame twist of the base origin, linear part
// first; its tau is the body-frame wrench [force; moment]. The base rotation
// is the Hamilton rotation of the quaternion divided by its squared norm, so a
// non-unit quaternion is well defined. Gravity enters as a fictitious base
// acceleration a_0 = -g (the paper's a_g, read with that sign).
//
// Every routine is templated on the scalar; instantiating it with the
// counting type Cd tallies the arithmetic of one evaluation.

#include <array>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace orc {

// ---------------------------------------------------------------- counting
// The counting scalar tallies the arithmetic of one evaluation that depends
// on the robot's state. A value is "known" when it follows from the model
// alone (constants, model parameters and what is computed from them only):
// that work can be done once per model, so it is not counted. An operation
// with a known 0 operand (x + 0, x * 0) or a known +-1 factor (x * 1) is the
// trivial form of the plain algorithm's general step (an identity joint-origin
// rotation, a zero parent velocity at the root, the zero linear part of a
// revolute motion subspace) and is not counted either. Everything else counts
// once: add/sub, mul, div, sqrt and sin/cos separately. The values themselves
// are ordinary FP64, so results are unchanged.
struct Tally {
  long long addsub, mul, div, sqrt, trig;
};
static thread_local Tally g_tally = {0, 0, 0, 0, 0};

struct Cd {
  double v;
  bool known;  // determined by the model alone
  Cd() : v(0.0), known(true) {}
  Cd(double x) : v(x), known(true) {}  // constants and model parameters
  static Cd var(double x) { Cd c(x); c.known = false; return c; }  // a state input
};
inline Cd cd_res(double x, bool known) { Cd c(x); c.known = known; return c; }
inline bool is0(const Cd& a) { return a.known && a.v == 0.0; }
inline bool is1(const Cd& a) { return a.known && (a.v == 1.0 || a.v == -1.0); }
inline Cd operator+(Cd a, Cd b) {
  if (a.known && b.known) return Cd(a.v + b.v);
  if (is0(a)) return b;
  if (is0(b)) return a;
  ++g_tally.addsub;
  return cd_res(a.v + b.v, false);
}
inline Cd operator-(Cd a) { return cd_res(-a.v, a.known); }
inline Cd operator-(Cd a, Cd b) {
  if (a.known && b.known) return Cd(a.v - b.v);
  if (is0(b)) return a;
  if (is0(a)) return -b;
  ++g_tally.addsub;
  return cd_res(a.v - b.v, false);
}
inline Cd operator*(Cd a, Cd b) {
  if (a.known && b.known) return Cd(a.v * b.v);
  if (is0(a) || is0(b)) return Cd(0.0);
  if (is1(a)) return cd_res(a.v * b.v, b.known);
  if (is1(b)) return cd_res(a.v * b.v, a.known);
  ++g_tally.mul;
  return cd_res(a.v * b.v, false);
}
inline Cd operator/(Cd a, Cd b) {
  if (a.known && b.known) return Cd(a.v / b.v);
  if (is0(a)) return Cd(0.0);
  if (is1(b)) return cd_res(a.v / b.v, a.known);
  ++g_tally.div;
  return cd_res(a.v / b.v, false);
}
inline Cd& operator+=(Cd& a, Cd b) { a = a + b; return a; }
inline Cd& operator-=(Cd& a, Cd b) { a = a - b; return a; }
inline Cd& operator*=(Cd& a, Cd b) { a = a * b; return a; }
inline Cd& operator/=(Cd& a, Cd b) { a = a / b; return a; }
inline Cd sqrt(Cd a) {
  if (!a.known) ++g_tally.sqrt;
  return cd_res(std::sqrt(a.v), a.known);
}
inline Cd sin(Cd a) {
  if (!a.known) ++g_tally.trig;
  return cd_res(std::sin(a.v), a.known);
}
inline Cd cos(Cd a) {
  if (!a.known) ++g_tally.trig;
  return cd_res(std::cos(a.v), a.known);
}
inline double val(Cd a) { return a.v; }
inline double val(double a) { return a; }

// ---------------------------------------------------------------- 3-D algebra
template <class T> using V3 = std::array<T, 3>;
template <class T> using M3 = std::array<T, 9>;  // row-major

template <class T> V3<T> add(const V3<T>& a, const V3<T>& b) { return {a[0] + b[0], a[1] + b[1], a[2] + b[2]}; }
template <class T> V3<T> sub(const V3<T>& a, const V3<T>& b) { return {a[0] - b[0], a[1] - b[1], a[2] - b[2]}; }
template <class T> V3<T> scl(const T& s, const V3<T>& a) { return {s * a[0], s * a[1], s * a[2]}; }
template <class T> T dot(const V3<T>& a, const V3<T>& b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
template <class T> V3<T> cross(const V3<T>& a, const V3<T>& b) {
  return {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
}
template <class T> V3<T> mv(const M3<T>& A, const V3<T>& x) {  // A x
  return {A[0] * x[0] + A[1] * x[1] + A[2] * x[2], A[3] * x[0] + A[4] * x[1] + A[5] * x[2],
          A[6] * x[0] + A[7] * x[1] + A[8] * x[2]};
}
template <class T> V3<T> mtv(const M3<T>& A, const V3<T>& x) {  // A^T x
  return {A[0] * x[0] + A[3] * x[1] + A[6] * x[2], A[1] * x[0] + A[4] * x[1] + A[7] * x[2],
          A[2] * x[0] + A[5] * x[1] + A[8] * x[2]};
}
template <class T> M3<T> mm(const M3<T>& A, const M3<T>& B) {  // A B
  M3<T> C;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) C[3 * i + j] = A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j] + A[3 * i + 2] * B[6 + j];
  return C;
}
template <class T> M3<T> mtm(const M3<T>& A, const M3<T>& B) {  // A^T B
  M3<T> C;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) C[3 * i + j] = A[i] * B[j] + A[3 + i] * B[3 + j] + A[6 + i] * B[6 + j];
  return C;
}
template <class T> M3<T> madd(const M3<T>& A, const M3<T>& B) {
  M3<T> C;
  for (int k = 0; k < 9; ++k) C[k] = A[k] + B[k];
  return C;
}
template <class T> M3<T> msub(const M3<T>& A, const M3<T>& B) {
  M3<T> C;
  for (int k = 0; k < 9; ++k) C[k] = A[k] - B[k];
  return C;
}
// [a]x [b]x = b a^T - (a . b) 1
template <class T> M3<T> skew_skew(const V3<T>& a, const V3<T>& b) {
  T d = dot(a, b);
  M3<T> C;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) C[3 * i + j] = b[i] * a[j];
  C[0] = C[0] - d; C[4] = C[4] - d; C[8] = C[8] - d;
  return C;
}

// Rotation by angle q about the unit axis a (Rodrigues): c 1 + s [a]x + (1-c) a a^T.
template <class T> M3<T> rodrigues(const V3<double>& a, const T& q) {
  using std::cos; using std::sin;
  T c = cos(q), s = sin(q);
  T t = T(1.0) - c;
  M3<T> R;
  R[0] = c + t * (a[0] * a[0]);          R[1] = t * (a[0] * a[1]) - s * a[2];  R[2] = t * (a[0] * a[2]) + s * a[1];
  R[3] = t * (a[1] * a[0]) + s * a[2];   R[4] = c + t * (a[1] * a[1]);         R[5] = t * (a[1] * a[2]) - s * a[0];
  R[6] = t * (a[2] * a[0]) - s * a[1];   R[7] = t * (a[2] * a[1]) + s * a[0];  R[8] = c + t * (a[2] * a[2]);
  return R;
}

// Hamilton rotation of (w,x,y,z) divided by w^2+x^2+y^2+z^2.
template <class T> M3<T> quat_rot(const T& w, const T& x, const T& y, const T& z) {
  T ww = w * w, xx = x * x, yy = y * y, zz = z * z;
  T s = ww + xx + yy + zz;
  T xy = x * y, xz = x * z, yz = y * z, wx = w * x, wy = w * y, wz = w * z;
  M3<T> N = {ww + xx - yy - zz, T(2.0) * (xy - wz), T(2.0) * (xz + wy),
             T(2.0) * (xy + wz), ww - xx + yy - zz, T(2.0) * (yz - wx),
             T(2.0) * (xz - wy), T(2.0) * (yz + wx), ww - xx - yy + zz};
  for (int k = 0; k < 9; ++k) N[k] = N[k] / s;
  return N;
}

// ---------------------------------------------------------------- spatial algebra
// Motion [w; v] and force [n; f] vectors share the storage type.
template <class T> struct SV {
  V3<T> a, l;  // angular part, linear part
};
template <class T> SV<T> zero_sv() { return {V3<T>{T(0.0), T(0.0), T(0.0)}, V3<T>{T(0.0), T(0.0), T(0.0)}}; }
template <class T> SV<T> sadd(const SV<T>& x, const SV<T>& y) { return {add(x.a, y.a), add(x.l, y.l)}; }
template <class T> SV<T> ssub(const SV<T>& x, const SV<T>& y) { return {sub(x.a, y.a), sub(x.l, y.l)}; }
template <class T> SV<T> sscl(const T& s, const SV<T>& x) { return {scl(s, x.a), scl(s, x.l)}; }
template <class T> T sdot(const SV<T>& x, const SV<T>& y) { return dot(x.a, y.a) + dot(x.l, y.l); }
// motion cross motion: [w; v] x [w2; v2] = [w x w2; w x v2 + v x w2]
template <class T> SV<T> crm(const SV<T>& m, const SV<T>& x) {
  return {cross(m.a, x.a), add(cross(m.a, x.l), cross(m.l, x.a))};
}
// motion cross force: [w; v] x* [n; f] = [w x n + v x f; w x f]
template <class T> SV<T> crf(const SV<T>& m, const SV<T>& f) {
  return {add(cross(m.a, f.a), cross(m.l, f.l)), cross(m.a, f.l)};
}

// Plucker transform B_X_A: B is rotated by E (B coords = E * A coords) and its
// origin sits at r in A coordinates.
template <class T> struct PX {
  M3<T> E;
  V3<T> r;
};
// motion A -> B
template <class T> SV<T> xm(const PX<T>& X, const SV<T>& m) {
  return {mv(X.E, m.a), mv(X.E, sub(m.l, cross(X.r, m.a)))};
}
// force B -> A (the transpose of the motion transform)
template <class T> SV<T> xtf(const PX<T>& X, const SV<T>& f) {
  V3<T> fa = mtv(X.E, f.l);
  return {add(mtv(X.E, f.a), cross(X.r, fa)), fa};
}

// Rigid-body inertia about the frame origin: mass m, first moment h = m c,
// rotational inertia Ibar about the origin.
template <class T> struct RBI {
  T m;
  V3<T> h;
  M3<T> I;
};
template <class T> SV<T> imul(const RBI<T>& I, const SV<T>& x) {
  return {add(mv(I.I, x.a), cross(I.h, x.l)), sub(scl(I.m, x.l), cross(I.h, x.a))};
}
template <class T> RBI<T> iadd(const RBI<T>& A, const RBI<T>& B) { return {A.m + B.m, add(A.h, B.h), madd(A.I, B.I)}; }
// A_X*_B I B_X_A: the inertia given in B coordinates expressed in A coordinates.
// m' = m, h' = E^T h + m r, I' = E^T I E - [r]x[E^T h]x - [h']x[r]x.
template <class T> RBI<T> xtix(const PX<T>& X, const RBI<T>& I) {
  V3<T> Eh = mtv(X.E, I.h);
  V3<T> h2 = add(Eh, scl(I.m, X.r));
  M3<T> R = mm(mtm(X.E, I.I), X.E);
  R = msub(R, skew_skew(X.r, Eh));
  R = msub(R, skew_skew(h2, X.r));
  return {I.m, h2, R};
}

// ---------------------------------------------------------------- model
struct Model {
  int n = 0, nq = 0, nv = 0;
  bool floating = false;
  std::vector<int> parent, jtype, nqi, nvi, qofs, vofs;
  std::vector<V3<double>> axis, p;
  std::vector<M3<double>> Rfix;
  std::vector<RBI<double>> I;  // about the body origin
  V3<double> g{0.0, 0.0, 0.0};
};

template <class T> RBI<T> cvt(const RBI<double>& I) {
  RBI<T> o;
  o.m = T(I.m);
  for (int k = 0; k < 3; ++k) o.h[k] = T(I.h[k]);
  for (int k = 0; k < 9; ++k) o.I[k] = T(I.I[k]);
  return o;
}

// Joint transform i_X_parent(i) for body i.
template <class T> PX<T> jcalc(const Model& M, int i, const T* q) {
  PX<T> X;
  if (M.jtype[i] == 1) {
    const T* qb = q + M.qofs[i];
    M3<T> R = quat_rot(qb[3], qb[4], qb[5], qb[6]);  // base axes in world coords
    for (int k = 0; k < 9; ++k) X.E[k] = R[3 * (k % 3) + k / 3];  // E = R^T
    X.r = {qb[0], qb[1], qb[2]};
  } else {
    M3<T> RJ = rodrigues(M.axis[i], q[M.qofs[i]]);
    M3<T> Rf;
    for (int k = 0; k < 9; ++k) Rf[k] = T(M.Rfix[i][k]);
    M3<T> R = mm(Rf, RJ);  // child axes in parent coords
    for (int k = 0; k < 9; ++k) X.E[k] = R[3 * (k % 3) + k / 3];
    X.r = {T(M.p[i][0]), T(M.p[i][1]), T(M.p[i][2])};
  }
  return X;
}

// Column k of the motion subspace S_i (body coordinates).
template <class T> SV<T> scol(const Model& M, int i, int k) {
  SV<T> s = zero_sv<T>();
  if (M.jtype[i] == 1) {
    if (k < 3) s.l[k] = T(1.0); else s.a[k - 3] = T(1.0);  // qd = [v; w]
  } else {
    s.a = {T(M.axis[i][0]), T(M.axis[i][1]), T(M.axis[i][2])};
  }
  return s;
}
// S_i x for the joint's generalized velocity block x.
template <class T> SV<T> smul(const Model& M, int i, const T* x) {
  if (M.jtype[i] == 1) return {V3<T>{x[3], x[4], x[5]}, V3<T>{x[0], x[1], x[2]}};
  return {scl(x[0], V3<T>{T(M.axis[i][0]), T(M.axis[i][1]), T(M.axis[i][2])}), V3<T>{T(0.0), T(0.0), T(0.0)}};
}
// S_i^T f written to out[0..nv_i).
template <class T> void stmul(const Model& M, int i, const SV<T>& f, T* out) {
  if (M.jtype[i] == 1) {
    for (int k = 0; k < 3; ++k) { out[k] = f.l[k]; out[3 + k] = f.a[k]; }
  } else {
    out[0] = dot(f.a, V3<T>{T(M.axis[i][0]), T(M.axis[i][1]), T(M.axis[i][2])});
  }
}

template <class T> SV<T> gravity_acc(const Model& M) {  // a_0 = -g, world frame
  SV<T> a = zero_sv<T>();
  for (int k = 0; k < 3; ++k) a.l[k] = T(-M.g[k]);
  return a;
}

// ---------------------------------------------------------------- kinematics
// World pose of every body: R (body axes in world coords), p (origin).
template <class T> void fk(const Model& M, const T* q, std::vector<M3<T>>& Rw, std::vector<V3<T>>& pw) {
  Rw.resize(M.n); pw.resize(M.n);
  for (int i = 0; i < M.n; ++i) {
    PX<T> X = jcalc(M, i, q);
    M3<T> R;  // body axes in parent coords = E^T
    for (int k = 0; k < 9; ++k) R[k] = X.E[3 * (k % 3) + k / 3];
    int l = M.parent[i];
    if (l < 0) { Rw[i] = R; pw[i] = X.r; }
    else { Rw[i] = mm(Rw[l], R); pw[i] = add(pw[l], mv(Rw[l], X.r)); }
  }
}

// World-aligned geometric Jacobian of body frame k at its origin: rows [v; w].
template <class T> void jacobian(const Model& M, const T* q, int k, T* J /*6 x nv row-major*/) {
  std::vector<M3<T>> Rw; std::vector<V3<T>> pw;
  fk(M, q, Rw, pw);
  for (int e = 0; e < 6 * M.nv; ++e) J[e] = T(0.0);
  for (int j = k; j >= 0; j = M.parent[j]) {
    int c0 = M.vofs[j];
    if (M.jtype[j] == 1) {
      V3<T> d = sub(pw[k], pw[j]);
      for (int c = 0; c < 3; ++c) {
        V3<T> Rc = {Rw[j][c], Rw[j][3 + c], Rw[j][6 + c]};  // column c of R
        // linear velocity part of the base twist: v_k = R v_B + (R w_B) x d
        for (int r = 0; r < 3; ++r) J[r * M.nv + c0 + c] = Rc[r];
        V3<T> w = cross(Rc, d);
        for (int r = 0; r < 3; ++r) {
          J[r * M.nv + c0 + 3 + c] = w[r];
          J[(3 + r) * M.nv + c0 + 3 + c] = Rc[r];
        }
      }
    } else {
      V3<T> z = mv(Rw[j], V3<T>{T(M.axis[j][0]), T(M.axis[j][1]), T(M.axis[j][2])});
      V3<T> w = cross(z, sub(pw[k], pw[j]));
      for (int r = 0; r < 3; ++r) {
        J[r * M.nv + c0] = w[r];
        J[(3 + r) * M.nv + c0] = z[r];
      }
    }
  }
}

// ---------------------------------------------------------------- external forces
// External spatial force on body i, given in world axes as [force f; moment n
// about the world origin] (fext + 6 i), expressed in body i's coordinates:
// [R^T (n - p x f); R^T f] with (R, p) the body's world pose (Alg. 1 takes
// the forces in the root frame; the recursion here works in body frames).
template <class T> SV<T> fext_body(const M3<T>& Rw, const V3<T>& pw, const T* fe) {
  const V3<T> f = {fe[0], fe[1], fe[2]}, n = {fe[3], fe[4], fe[5]};
  return {mtv(Rw, sub(n, cross(pw, f))), mtv(Rw, f)};
}

// ---------------------------------------------------------------- RNEA
// tau = ID(q, qd, qdd) - sum_i J_i^T F_ext,i; qdd == nullptr means qdd = 0
// (bias force h(q, qd)), fext == nullptr means no external forces. Body i's
// force balance subtracts the external force, as in Alg. 1.
// Xin, when given, holds every body's joint transform already built from q
// (forward dynamics builds them once for RNEA and CRBA).
template <class T> void rnea(const Model& M, const T* q, const T* qd, const T* qdd, T* tau,
                             const T* fext = nullptr, const std::vector<PX<T>>* Xin = nullptr) {
  const int n = M.n;
  std::vector<PX<T>> X(n);
  std::vector<SV<T>> v(n), a(n), f(n);
  std::vector<M3<T>> Rw;
  std::vector<V3<T>> pw;
  if (fext) fk(M, q, Rw, pw);
  const SV<T> a0 = gravity_acc<T>(M);
  for (int i = 0; i < n; ++i) {
    X[i] = Xin ? (*Xin)[i] : jcalc(M, i, q);
    int l = M.parent[i];
    SV<T> vJ = smul(M, i, qd + M.vofs[i]);
    SV<T> vp = l < 0 ? zero_sv<T>() : v[l];
    SV<T> ap = l < 0 ? a0 : a[l];
    v[i] = sadd(xm(X[i], vp), vJ);
    a[i] = sadd(xm(X[i], ap), crm(v[i], vJ));
    if (qdd) a[i] = sadd(a[i], smul(M, i, qdd + M.vofs[i]));
    RBI<T> I = cvt<T>(M.I[i]);
    f[i] = sadd(imul(I, a[i]), crf(v[i], imul(I, v[i])));
    if (fext) f[i] = ssub(f[i], fext_body(Rw[i], pw[i], fext + 6 * i));
  }
  for (int i = n - 1; i >= 0; --i) {
    stmul(M, i, f[i], tau + M.vofs[i]);
    int l = M.parent[i];
    if (l >= 0) f[l] = sadd(f[l], xtf(X[i], f[i]));
  }
}

// ---------------------------------------------------------------- CRBA
template <class T> void crba(const Model& M, const T* q, T* H /*nv x nv row-major*/,
                             const std::vector<PX<T>>* Xin = nullptr) {
  const int n = M.n, nv = M.nv;
  std::vector<PX<T>> X(n);
  std::vector<RBI<T>> Ic(n);
  for (int i = 0; i < n; ++i) { X[i] = Xin ? (*Xin)[i] : jcalc(M, i, q); Ic[i] = cvt<T>(M.I[i]); }
  for (int e = 0; e < nv * nv; ++e) H[e] = T(0.0);
  for (int i = n - 1; i >= 0; --i) {
    int l = M.parent[i];
    if (l >= 0) Ic[l] = iadd(Ic[l], xtix(X[i], Ic[i]));
  }
  for (int i = 0; i < n; ++i) {
    for (int ci = 0; ci < M.nvi[i]; ++ci) {
      SV<T> F = imul(Ic[i], scol<T>(M, i, ci));
      int r = M.vofs[i] + ci;
      for (int cj = 0; cj < M.nvi[i]; ++cj) {
        T hij = sdot(F, scol<T>(M, i, cj));
        H[r * nv + M.vofs[i] + cj] = hij;
      }
      for (int j = i; M.parent[j] >= 0;) {
        F = xtf(X[j], F);
        j = M.parent[j];
        for (int cj = 0; cj < M.nvi[j]; ++cj) {
          T hij = sdot(F, scol<T>(M, j, cj));
          H[r * nv + M.vofs[j] + cj] = hij;
          H[(M.vofs[j] + cj) * nv + r] = hij;
        }
      }
    }
  }
}

// ---------------------------------------------------------------- factorisations
// Dense M = L L^T (no pivoting), then x = M^-1 b in place.
template <class T> void chol_llt_solve(int n, T* H, T* b) {
  for (int j = 0; j < n; ++j) {
    T s = H[j * n + j];
    for (int k = 0; k < j; ++k) s = s - H[j * n + k] * H[j * n + k];
    using std::sqrt;
    T d = sqrt(s);
    H[j * n + j] = d;
    for (int i = j + 1; i < n; ++i) {
      T t = H[i * n + j];
      for (int k = 0; k < j; ++k) t = t - H[i * n + k] * H[j * n + k];
      H[i * n + j] = t / d;
    }
  }
  for (int i = 0; i < n; ++i) {  // L y = b
    T t = b[i];
    for (int k = 0; k < i; ++k) t = t - H[i * n + k] * b[k];
    b[i] = t / H[i * n + i];
  }
  for (int i = n - 1; i >= 0; --i) {  // L^T x = y
    T t = b[i];
    for (int k = i + 1; k < n; ++k) t = t - H[k * n + i] * b[k];
    b[i] = t / H[i * n + i];
  }
}

// Velocity-index parent: lam[k] is the closest ancestor DoF of DoF k.
inline std::vector<int> dof_parent(const Model& M) {
  std::vector<int> lam(M.nv);
  for (int i = 0; i < M.n; ++i) {
    int l = M.parent[i];
    int prev = l < 0 ? -1 : M.vofs[l] + M.nvi[l] - 1;
    for (int k = 0; k < M.nvi[i]; ++k) { lam[M.vofs[i] + k] = prev; prev = M.vofs[i] + k; }
  }
  return lam;
}

// Branch-sparse M = L^T L (RBDA Sec. 6.5): leaves to root, no fill-in, then
// x = M^-1 b = L^-1 L^-T b in place.
template <class T> void ltl_solve(int n, const std::vector<int>& lam, T* H, T* b) {
  using std::sqrt;
  for (int k = n - 1; k >= 0; --k) {
    H[k * n + k] = sqrt(H[k * n + k]);
    for (int i = lam[k]; i >= 0; i = lam[i]) H[k * n + i] = H[k * n + i] / H[k * n + k];
    for (int i = lam[k]; i >= 0; i = lam[i])
      for (int j = i; j >= 0; j = lam[j]) H[i * n + j] = H[i * n + j] - H[k * n + i] * H[k * n + j];
  }
  for (int k = n - 1; k >= 0; --k) {  // L^T y = b
    b[k] = b[k] / H[k * n + k];
    for (int i = lam[k]; i >= 0; i = lam[i]) b[i] = b[i] - H[k * n + i] * b[k];
  }
  for (int k = 0; k < n; ++k) {  // L x = y
    for (int i = lam[k]; i >= 0; i = lam[i]) b[k] = b[k] - H[k * n + i] * b[i];
    b[k] = b[k] / H[k * n + k];
  }
}

// ---------------------------------------------------------------- ABA
// General symmetric 6x6 articulated inertias, stored dense [ang; lin] order.
template <class T> using M6 = std::array<T, 36>;
template <class T> M6<T> rbi_dense(const RBI<T>& I) {
  M6<T> A;
  // [Ibar, [h]x; [h]x^T, m 1]
  M3<T> hx = {T(0.0), -I.h[2], I.h[1], I.h[2], T(0.0), -I.h[0], -I.h[1], I.h[0], T(0.0)};
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      A[6 * r + c] = I.I[3 * r + c];
      A[6 * r + 3 + c] = hx[3 * r + c];
      A[6 * (3 + r) + c] = hx[3 * c + r];
      A[6 * (3 + r) + 3 + c] = (r == c) ? I.m : T(0.0);
    }
  return A;
}
template <class T> SV<T> m6v(const M6<T>& A, const SV<T>& x) {
  T in[6] = {x.a[0], x.a[1], x.a[2], x.l[0], x.l[1], x.l[2]};
  T o[6];
  for (int r = 0; r < 6; ++r) {
    T s = A[6 * r] * in[0];
    for (int c = 1; c < 6; ++c) s = s + A[6 * r + c] * in[c];
    o[r] = s;
  }
  return {V3<T>{o[0], o[1], o[2]}, V3<T>{o[3], o[4], o[5]}};
}
template <class T> M6<T> px_dense(const PX<T>& X) {  // motion transform [E 0; -E[r]x E]
  M6<T> A;
  M3<T> rx = {T(0.0), -X.r[2], X.r[1], X.r[2], T(0.0), -X.r[0], -X.r[1], X.r[0], T(0.0)};
  M3<T> Erx = mm(X.E, rx);
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      A[6 * r + c] = X.E[3 * r + c];
      A[6 * r + 3 + c] = T(0.0);
      A[6 * (3 + r) + c] = -Erx[3 * r + c];
      A[6 * (3 + r) + 3 + c] = X.E[3 * r + c];
    }
  return A;
}
template <class T> M6<T> xtax(const PX<T>& X, const M6<T>& A) {  // X^T A X
  M6<T> P = px_dense(X), AX, O;
  for (int r = 0; r < 6; ++r)
    for (int c = 0; c < 6; ++c) {
      T s = A[6 * r] * P[c];
      for (int k = 1; k < 6; ++k) s = s + A[6 * r + k] * P[6 * k + c];
      AX[6 * r + c] = s;
    }
  for (int r = 0; r < 6; ++r)
    for (int c = 0; c < 6; ++c) {
      T s = P[r] * AX[c];
      for (int k = 1; k < 6; ++k) s = s + P[6 * k + r] * AX[6 * k + c];
      O[6 * r + c] = s;
    }
  return O;
}

// Solve the small dense SPD system D x = b (size m <= 6) by L L^T.
template <class T> void small_spd_solve(int m, T* D, T* b) { chol_llt_solve(m, D, b); }

template <class T> void aba(const Model& M, const T* q, const T* qd, const T* tau, T* qdd, const T* fext = nullptr) {
  const int n = M.n;
  std::vector<PX<T>> X(n);
  std::vector<SV<T>> v(n), c(n), pA(n), a(n);
  std::vector<M3<T>> Rw;
  std::vector<V3<T>> pw;
  if (fext) fk(M, q, Rw, pw);
  std::vector<M6<T>> IA(n);
  std::vector<std::vector<SV<T>>> U(n);
  std::vector<std::vector<T>> D(n), u(n);
  for (int i = 0; i < n; ++i) {
    X[i] = jcalc(M, i, q);
    int l = M.parent[i];
    SV<T> vJ = smul(M, i, qd + M.vofs[i]);
    v[i] = sadd(l < 0 ? zero_sv<T>() : xm(X[i], v[l]), vJ);
    c[i] = crm(v[i], vJ);
    RBI<T> I = cvt<T>(M.I[i]);
    IA[i] = rbi_dense(I);
    pA[i] = crf(v[i], imul(I, v[i]));
    if (fext) pA[i] = ssub(pA[i], fext_body(Rw[i], pw[i], fext + 6 * i));
  }
  for (int i = n - 1; i >= 0; --i) {
    const int m = M.nvi[i];
    U[i].resize(m); D[i].assign(m * m, T(0.0)); u[i].assign(m, T(0.0));
    for (int k = 0; k < m; ++k) U[i][k] = m6v(IA[i], scol<T>(M, i, k));
    for (int r = 0; r < m; ++r)
      for (int k = 0; k < m; ++k) D[i][r * m + k] = sdot(scol<T>(M, i, r), U[i][k]);
    std::vector<T> stp(m);
    stmul(M, i, pA[i], stp.data());
    for (int k = 0; k < m; ++k) u[i][k] = tau[M.vofs[i] + k] - stp[k];
    int l = M.parent[i];
    if (l >= 0) {
      // Dinv U^T and Dinv u via small solves
      std::vector<T> Dc(D[i]);
      std::vector<T> Dinv_u(u[i]);
      small_spd_solve(m, Dc.data(), Dinv_u.data());
      M6<T> Ia = IA[i];
      // Ia -= U Dinv U^T, built column by column
      for (int k = 0; k < m; ++k) {
        std::vector<T> e(m, T(0.0));
        e[k] = T(1.0);
        std::vector<T> Dk(D[i]);
        small_spd_solve(m, Dk.data(), e.data());  // column k of Dinv
        for (int r = 0; r < 6; ++r)
          for (int cc = 0; cc < 6; ++cc) {
            T ur = r < 3 ? U[i][k].a[r] : U[i][k].l[r - 3];
            T s = T(0.0);
            for (int kk = 0; kk < m; ++kk) {
              T uc = cc < 3 ? U[i][kk].a[cc] : U[i][kk].l[cc - 3];
              s = s + e[kk] * uc;
            }
            Ia[6 * r + cc] = Ia[6 * r + cc] - ur * s;
          }
      }
      SV<T> pa = sadd(pA[i], m6v(Ia, c[i]));
      for (int k = 0; k < m; ++k) pa = sadd(pa, sscl(Dinv_u[k], U[i][k]));
      IA[l] = [&] { M6<T> t = xtax(X[i], Ia); M6<T> o; for (int e = 0; e < 36; ++e) o[e] = IA[l][e] + t[e]; return o; }();
      pA[l] = sadd(pA[l], xtf(X[i], pa));
    }
  }
  const SV<T> a0 = gravity_acc<T>(M);
  for (int i = 0; i < n; ++i) {
    const int m = M.nvi[i];
    int l = M.parent[i];
    SV<T> ap = sadd(xm(X[i], l < 0 ? a0 : a[l]), c[i]);
    std::vector<T> rhs(m);
    for (int k = 0; k < m; ++k) rhs[k] = u[i][k] - sdot(U[i][k], ap);
    std::vector<T> Dc(D[i]);
    small_spd_solve(m, Dc.data(), rhs.data());
    for (int k = 0; k < m; ++k) qdd[M.vofs[i] + k] = rhs[k];
    a[i] = sadd(ap, smul(M, i, rhs.data()));
  }
}

// qdd = M^-1 (tau - h); method 0: dense L L^T, 1: branch-sparse L^T L, 2: ABA.
// With external forces (fext non-null) h includes -sum_i J_i^T F_ext,i.
template <class T> void fwd_dyn(const Model& M, const T* q, const T* qd, const T* tau, T* qdd, int method,
                                const T* fext = nullptr) {
  const int nv = M.nv;
  if (method == 2) { aba(M, q, qd, tau, qdd, fext); return; }
  std::vector<T> h(nv), H(nv * nv);
  std::vector<PX<T>> X(M.n);  // joint transforms, built once for both passes
  for (int i = 0; i < M.n; ++i) X[i] = jcalc(M, i, q);
  rnea(M, q, qd, (const T*)nullptr, h.data(), fext, &X);
  crba(M, q, H.data(), &X);
  for (int k = 0; k < nv; ++k) qdd[k] = tau[k] - h[k];
  if (method == 0) chol_llt_solve(nv, H.data(), qdd);
  else ltl_solve(nv, dof_parent(M), H.data(), qdd);
}

}  // namespace orc

// ================================================================ C ABI
using namespace orc;

extern "C" {

struct orc_model {
  int32_t n_bodies;
  const int32_t* parent;
  const int32_t* joint_type;
  const double* axis;
  const double* origin;
  const double* mass;
  const double* com;
  const double* inertia;
  double gravity[3];
};

}  // extern "C"

static int build_model(const orc_model* d, Model& M) {
  if (!d || d->n_bodies <= 0) return 1;
  const int n = d->n_bodies;
  M.n = n;
  M.parent.assign(d->parent, d->parent + n);
  M.jtype.assign(d->joint_type, d->joint_type + n);
  M.nqi.resize(n); M.nvi.resize(n); M.qofs.resize(n); M.vofs.resize(n);
  M.axis.resize(n); M.p.resize(n); M.Rfix.resize(n); M.I.resize(n);
  int qo = 0, vo = 0;
  for (int i = 0; i < n; ++i) {
    if (M.parent[i] >= i) return 1;
    if (M.jtype[i] == 1 && i != 0) return 1;
    M.nqi[i] = M.jtype[i] == 1 ? 7 : 1;
    M.nvi[i] = M.jtype[i] == 1 ? 6 : 1;
    M.qofs[i] = qo; M.vofs[i] = vo;
    qo += M.nqi[i]; vo += M.nvi[i];
    // The axis is given as a direction; it is normalised here (an FP32-rounded
    // unit vector is off by ~6e-8, enough to make R(q) measurably non-orthogonal).
    const double* ax = d->axis + 3 * i;
    const double an = std::sqrt(ax[0] * ax[0] + ax[1] * ax[1] + ax[2] * ax[2]);
    if (M.jtype[i] == 0 && !(an > 0.0)) return 1;
    for (int k = 0; k < 3; ++k) { M.axis[i][k] = an > 0.0 ? ax[k] / an : 0.0; M.p[i][k] = d->origin[12 * i + 9 + k]; }
    for (int k = 0; k < 9; ++k) M.Rfix[i][k] = d->origin[12 * i + k];
    const double m = d->mass[i];
    const double* c = d->com + 3 * i;
    const double* J = d->inertia + 6 * i;  // xx yy zz xy xz yz about the CoM
    M3<double> Ic = {J[0], J[3], J[4], J[3], J[1], J[5], J[4], J[5], J[2]};
    // about the origin: Ic + m (|c|^2 1 - c c^T)
    const double cc = c[0] * c[0] + c[1] * c[1] + c[2] * c[2];
    RBI<double> I;
    I.m = m;
    I.h = {m * c[0], m * c[1], m * c[2]};
    for (int r = 0; r < 3; ++r)
      for (int s = 0; s < 3; ++s) I.I[3 * r + s] = Ic[3 * r + s] + m * ((r == s ? cc : 0.0) - c[r] * c[s]);
    M.I[i] = I;
  }
  M.nq = qo; M.nv = vo;
  M.floating = M.jtype[0] == 1;
  for (int k = 0; k < 3; ++k) M.g[k] = d->gravity[k];
  return 0;
}

extern "C" {

int orc_dims(const orc_model* d, int* nq, int* nv) {
  Model M;
  if (build_model(d, M)) return 1;
  *nq = M.nq; *nv = M.nv;
  return 0;
}

int orc_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

// Threads for the following calls (n >= 1); returns the previous count.
int orc_set_threads(int n) {
#ifdef _OPENMP
  const int old = omp_get_max_threads();
  if (n >= 1) omp_set_num_threads(n);
  return old;
#else
  (void)n;
  return 1;
#endif
}

// All arrays are instance-major double: q [B][nq], qd/qdd/tau [B][nv].
int orc_fk(const orc_model* d, int64_t B, const double* q, double* T /*[B][n][12]*/) {
  Model M;
  if (build_model(d, M)) return 1;
#pragma omp parallel for schedule(static)
  for (int64_t b = 0; b < B; ++b) {
    std::vector<M3<double>> Rw; std::vector<V3<double>> pw;
    fk(M, q + b * M.nq, Rw, pw);
    double* o = T + b * M.n * 12;
    for (int i = 0; i < M.n; ++i) {
      for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) o[12 * i + 4 * r + c] = Rw[i][3 * r + c];
        o[12 * i + 4 * r + 3] = pw[i][r];
      }
    }
  }
  return 0;
}

int orc_jacobian(const orc_model* d, int64_t B, const double* q, int32_t nf, const int32_t* frames,
                 double* J /*[B][nf][6][nv]*/) {
  Model M;
  if (build_model(d, M)) return 1;
  for (int f = 0; f < nf; ++f)
    if (frames[f] < 0 || frames[f] >= M.n) return 1;
#pragma omp parallel for schedule(static)
  for (int64_t b = 0; b < B; ++b)
    for (int f = 0; f < nf; ++f) jacobian(M, q + b * M.nq, frames[f], J + (b * nf + f) * 6 * M.nv);
  return 0;
}

int orc_rnea(const orc_model* d, int64_t B, const double* q, const double* qd, const double* qdd, double* tau) {
  Model M;
  if (build_model(d, M)) return 1;
#pragma omp parallel for schedule(static)
  for (int64_t b = 0; b < B; ++b)
    rnea(M, q + b * M.nq, qd + b * M.nv, qdd ? qdd + b * M.nv : (const double*)nullptr, tau + b * M.nv);
  return 0;
}

// orc_rnea with external forces fext [B][n][6] (world axes: force, then
// moment about the world origin).
int orc_rnea_ext(const orc_model* d, int64_t B, const double* q, const double* qd, const double* qdd,
                 const double* fext, double* tau) {
  Model M;
  if (build_model(d, M) || !fext) return 1;
#pragma omp parallel for schedule(static)
  for (int64_t b = 0; b < B; ++b)
    rnea(M, q + b * M.nq, qd + b * M.nv, qdd ? qdd + b * M.nv : (const double*)nullptr, tau + b * M.nv,
         fext + b * 6 * M.n);
  return 0;
}

// Like orc_rnea with gravity switched off (c(q, qd) alone when qdd is null).
int orc_rnea_nograv(const orc_model* d, int64_t B, const double* q, const double* qd, const double* qdd,
                    double* tau) {
  Model M;
  if (build_model(d, M)) return 1;
  M.g = {0.0, 0.0, 0.0};
#pragma omp parallel for schedule(static)
  for (int64_t b = 0; b < B; ++b)
    rnea(M, q + b * M.nq, qd + b * M.nv, qdd ? qdd + b * M.nv : (const double*)nullptr, tau + b * M.nv);
  return 0;
}

int orc_crba(const orc_model* d, int64_t B, const double* q, double* H /*[B][nv][nv]*/) {
  Model M;
  if (build_model(d, M)) return 1;
#pragma omp parallel for schedule(static)
  for (int64_t b = 0; b < B; ++b) crba(M, q + b * M.nq, H + b * M.nv * M.nv);
  return 0;
}

int orc_fwd_dyn(const orc_model* d, int64_t B, const double* q, const double* qd, const double* tau, double* qdd,
                int method) {
  Model M;
  if (build_model(d, M) || method < 0 || method > 2) return 1;
#pragma omp parallel for schedule(static)
  for (int64_t b = 0; b < B; ++b)
    fwd_dyn(M, q + b * M.nq, qd + b * M.nv, tau + b * M.nv, qdd + b * M.nv, method);
  return 0;
}

int orc_fwd_dyn_ext(const orc_model* d, int64_t B, const double* q, const double* qd, const double* tau,
                    const double* fext, double* qdd, int method) {
  Model M;
  if (build_model(d, M) || method < 0 || method > 2 || !fext) return 1;
#pragma omp parallel for schedule(static)
  for (int64_t b = 0; b < B; ++b)
    fwd_dyn(M, q + b * M.nq, qd + b * M.nv, tau + b * M.nv, qdd + b * M.nv, method, fext + b * 6 * M.n);
  return 0;
}

// Jacobian-vector product of qdd = FD(q, qd, tau, F) along the tangent (dq,
// dqd, dtau, dF), the directional derivative by one central difference of
// step h: [FD(x + h dx) - FD(x - h dx)] / 2h (raw quaternion components are
// moved like any other coordinate). fext (external forces, [B][6n]) and dfext
// may be null (none, and a zero tangent).
int orc_fwd_dyn_jvp_fd(const orc_model* d, int64_t B, const double* q, const double* qd, const double* tau,
                       const double* fext, const double* dq, const double* dqd, const double* dtau,
                       const double* dfext, double* dqdd, double h, int method) {
  Model M;
  if (build_model(d, M) || method < 0 || method > 2) return 1;
  const int nq = M.nq, nv = M.nv, nf = 6 * M.n;
  const bool ext = fext || dfext;
#pragma omp parallel for schedule(static)
  for (int64_t b = 0; b < B; ++b) {
    std::vector<double> xp(nq), xm(nq), yp(nv), ym(nv), zp(nv), zm(nv), ap(nv), am(nv), fp(nf), fm(nf);
    for (int k = 0; k < nq; ++k) {
      xp[k] = q[b * nq + k] + h * dq[b * nq + k];
      xm[k] = q[b * nq + k] - h * dq[b * nq + k];
    }
    for (int k = 0; k < nv; ++k) {
      yp[k] = qd[b * nv + k] + h * dqd[b * nv + k];
      ym[k] = qd[b * nv + k] - h * dqd[b * nv + k];
      zp[k] = tau[b * nv + k] + h * dtau[b * nv + k];
      zm[k] = tau[b * nv + k] - h * dtau[b * nv + k];
    }
    for (int k = 0; k < nf && ext; ++k) {
      const double f0 = fext ? fext[b * nf + k] : 0.0, df = dfext ? dfext[b * nf + k] : 0.0;
      fp[k] = f0 + h * df;
      fm[k] = f0 - h * df;
    }
    fwd_dyn(M, xp.data(), yp.data(), zp.data(), ap.data(), method, ext ? fp.data() : nullptr);
    fwd_dyn(M, xm.data(), ym.data(), zm.data(), am.data(), method, ext ? fm.data() : nullptr);
    for (int k = 0; k < nv; ++k) dqdd[b * nv + k] = (ap[k] - am[k]) / (2.0 * h);
  }
  return 0;
}

// Jacobian-vector product of inverse dynamics tau = ID(q, qd, qdd, F) along
// (dq, dqd, dqdd, dF): one central difference of step h (raw quaternion
// components perturbed like any other coordinate). fext and dfext may be null.
int orc_rnea_jvp_fd(const orc_model* d, int64_t B, const double* q, const double* qd, const double* qdd,
                    const double* fext, const double* dq, const double* dqd, const double* dqdd,
                    const double* dfext, double* dtau, double h) {
  Model M;
  if (build_model(d, M)) return 1;
  const int nq = M.nq, nv = M.nv, nf = 6 * M.n;
  const bool ext = fext || dfext;
#pragma omp parallel for schedule(static)
  for (int64_t b = 0; b < B; ++b) {
    std::vector<double> xp(nq), xm(nq), yp(nv), ym(nv), zp(nv), zm(nv), tp(nv), tm(nv), fp(nf), fm(nf);
    for (int k = 0; k < nq; ++k) {
      xp[k] = q[b * nq + k] + h * dq[b * nq + k];
      xm[k] = q[b * nq + k] - h * dq[b * nq + k];
    }
    for (int k = 0; k < nv; ++k) {
      yp[k] = qd[b * nv + k] + h * dqd[b * nv + k];
      ym[k] = qd[b * nv + k] - h * dqd[b * nv + k];
      zp[k] = qdd[b * nv + k] + h * dqdd[b * nv + k];
      zm[k] = qdd[b * nv + k] - h * dqdd[b * nv + k];
    }
    for (int k = 0; k < nf && ext; ++k) {
      const double f0 = fext ? fext[b * nf + k] : 0.0, df = dfext ? dfext[b * nf + k] : 0.0;
      fp[k] = f0 + h * df;
      fm[k] = f0 - h * df;
    }
    rnea(M, xp.data(), yp.data(), zp.data(), tp.data(), ext ? fp.data() : (const double*)nullptr);
    rnea(M, xm.data(), ym.data(), zm.data(), tm.data(), ext ? fm.data() : (const double*)nullptr);
    for (int k = 0; k < nv; ++k) dtau[b * nv + k] = (tp[k] - tm[k]) / (2.0 * h);
  }
  return 0;
}

// Vector-Jacobian product of inverse dynamics tau = ID(q, qd, qdd, F) with
// cotangent lam: g_x = lam^T dID/dx for x = q, qd, qdd and F, by central
// differences of step h on every coordinate (raw quaternion components and
// every external-force component included). fext may be null (no forces); any
// output may be null.
int orc_rnea_vjp_fd(const orc_model* d, int64_t B, const double* q, const double* qd, const double* qdd,
                    const double* fext, const double* lam, double* gq, double* gqd, double* gqdd, double* gfext,
                    double h) {
  Model M;
  if (build_model(d, M)) return 1;
  const int nq = M.nq, nv = M.nv, nf = 6 * M.n;
  const bool ext = fext || gfext;
#pragma omp parallel for schedule(static)
  for (int64_t b = 0; b < B; ++b) {
    std::vector<double> x(nq), y(nv), z(nv), f(nf, 0.0), tp(nv), tm(nv);
    const double* l = lam + b * nv;
    const double* F = ext ? f.data() : nullptr;
    std::memcpy(x.data(), q + b * nq, nq * sizeof(double));
    std::memcpy(y.data(), qd + b * nv, nv * sizeof(double));
    std::memcpy(z.data(), qdd + b * nv, nv * sizeof(double));
    if (fext) std::memcpy(f.data(), fext + b * nf, nf * sizeof(double));
    auto diff = [&](double* v, int k) {
      const double v0 = v[k];
      v[k] = v0 + h; rnea(M, x.data(), y.data(), z.data(), tp.data(), F);
      v[k] = v0 - h; rnea(M, x.data(), y.data(), z.data(), tm.data(), F);
      v[k] = v0;
      double s = 0.0;
      for (int c = 0; c < nv; ++c) s += l[c] * (tp[c] - tm[c]);
      return s / (2.0 * h);
    };
    if (gq)
      for (int k = 0; k < nq; ++k) gq[b * nq + k] = diff(x.data(), k);
    if (gqd)
      for (int k = 0; k < nv; ++k) gqd[b * nv + k] = diff(y.data(), k);
    if (gqdd)
      for (int k = 0; k < nv; ++k) gqdd[b * nv + k] = diff(z.data(), k);
    if (gfext)
      for (int k = 0; k < nf; ++k) gfext[b * nf + k] = diff(f.data(), k);
  }
  return 0;
}

// Vector-Jacobian product of qdd = FD(q, qd, tau, F) with cotangent gbar, by
// central differences of step h on every coordinate (raw quaternion
// components and every external-force component included). fext may be null
// (no forces); any output may be null.
int orc_fwd_dyn_vjp_fd(const orc_model* d, int64_t B, const double* q, const double* qd, const double* tau,
                       const double* fext, const double* gbar, double* gq, double* gqd, double* gtau,
                       double* gfext, double h, int method) {
  Model M;
  if (build_model(d, M) || method < 0 || method > 2) return 1;
  const int nq = M.nq, nv = M.nv, nf = 6 * M.n;
  const bool ext = fext || gfext;
#pragma omp parallel for schedule(static)
  for (int64_t b = 0; b < B; ++b) {
    std::vector<double> x(nq), y(nv), z(nv), f(nf, 0.0), qp(nv), qm(nv);
    const double* g = gbar + b * nv;
    const double* F = ext ? f.data() : nullptr;
    auto contract = [&](void) {
      double s = 0.0;
      for (int k = 0; k < nv; ++k) s += g[k] * (qp[k] - qm[k]);
      return s / (2.0 * h);
    };
    std::memcpy(x.data(), q + b * nq, nq * sizeof(double));
    std::memcpy(y.data(), qd + b * nv, nv * sizeof(double));
    std::memcpy(z.data(), tau + b * nv, nv * sizeof(double));
    if (fext) std::memcpy(f.data(), fext + b * nf, nf * sizeof(double));
    auto diff = [&](double* v, int k) {
      const double v0 = v[k];
      v[k] = v0 + h; fwd_dyn(M, x.data(), y.data(), z.data(), qp.data(), method, F);
      v[k] = v0 - h; fwd_dyn(M, x.data(), y.data(), z.data(), qm.data(), method, F);
      v[k] = v0;
      return contract();
    };
    if (gq)
      for (int k = 0; k < nq; ++k) gq[b * nq + k] = diff(x.data(), k);
    if (gqd)
      for (int k = 0; k < nv; ++k) gqd[b * nv + k] = diff(y.data(), k);
    if (gtau)
      for (int k = 0; k < nv; ++k) gtau[b * nv + k] = diff(z.data(), k);
    if (gfext)
      for (int k = 0; k < nf; ++k) gfext[b * nf + k] = diff(f.data(), k);
  }
  return 0;
}

// Arithmetic of one evaluation of an operation, counted with the counting
// scalar: out = {add/sub, mul, div, sqrt, sin+cos}. op: 0 fk, 1 jacobian of
// every body frame, 2 rnea with qdd, 3 rnea bias (qdd = 0), 4 crba,
// 5 fwd_dyn dense L L^T, 6 fwd_dyn branch-sparse L^T L, 7 aba.
int orc_count_ops(const orc_model* d, int op, long long* out) {
  Model M;
  if (build_model(d, M)) return 1;
  const int nq = M.nq, nv = M.nv;
  // a generic state: every input is a variable with a value that is neither 0 nor 1
  std::vector<Cd> q(nq, Cd::var(0.1)), qd(nv, Cd::var(0.2)), qdd(nv, Cd::var(0.3)), tau(nv, Cd::var(0.4)), o(nv);
  if (M.floating) { q[3] = Cd::var(0.9); q[4] = Cd::var(0.3); q[5] = Cd::var(-0.2); q[6] = Cd::var(0.25); }
  g_tally = {0, 0, 0, 0, 0};
  switch (op) {
    case 0: { std::vector<M3<Cd>> R; std::vector<V3<Cd>> p; fk(M, q.data(), R, p); break; }
    case 1: {
      // All frames share one FK pass; the per-frame column assembly is counted per frame.
      std::vector<M3<Cd>> R; std::vector<V3<Cd>> p; fk(M, q.data(), R, p);
      Tally t0 = g_tally;
      std::vector<Cd> J(6 * nv);
      long long add = 0, mul = 0;
      for (int k = 0; k < M.n; ++k) {
        g_tally = {0, 0, 0, 0, 0};
        jacobian(M, q.data(), k, J.data());
        Tally tk = g_tally;
        add += tk.addsub - t0.addsub; mul += tk.mul - t0.mul;  // minus its own FK pass
      }
      g_tally = t0; g_tally.addsub += add; g_tally.mul += mul;
      break;
    }
    case 2: rnea(M, q.data(), qd.data(), qdd.data(), o.data()); break;
    case 3: rnea(M, q.data(), qd.data(), (const Cd*)nullptr, o.data()); break;
    case 4: { std::vector<Cd> H(nv * nv); crba(M, q.data(), H.data()); break; }
    case 5: fwd_dyn(M, q.data(), qd.data(), tau.data(), o.data(), 0); break;
    case 6: fwd_dyn(M, q.data(), qd.data(), tau.data(), o.data(), 1); break;
    case 7: fwd_dyn(M, q.data(), qd.data(), tau.data(), o.data(), 2); break;
    default: return 1;
  }
  out[0] = g_tally.addsub; out[1] = g_tally.mul; out[2] = g_tally.div; out[3] = g_tally.sqrt; out[4] = g_tally.trig;
  return 0;
}

}  // extern "C"
