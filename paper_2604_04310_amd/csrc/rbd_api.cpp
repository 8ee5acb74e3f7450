// Host side of librbd.so: model validation, FP64 precomputation of the
// device tables, and the argument checks of every C entry point.
#include <hip/hip_runtime.h>

#include <array>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <initializer_list>
#include <vector>

#include "rbd_internal.hpp"

namespace rbd {

static thread_local char g_err[512] = "";

rbd_status fail(rbd_status s, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return s;
}
void clear_error() { g_err[0] = '\0'; }

// ---- small FP64 3x3 helpers (row-major)
using D9 = std::array<double, 9>;
static D9 matmul(const D9& A, const D9& B) {
  D9 C{};
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) C[3 * i + j] = A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j] + A[3 * i + 2] * B[6 + j];
  return C;
}
static D9 transpose(const D9& A) { return {A[0], A[3], A[6], A[1], A[4], A[7], A[2], A[5], A[8]}; }
static const D9 kEye = {1, 0, 0, 0, 1, 0, 0, 0, 1};

// A rotation whose third column is the unit vector a (joint-aligned axes).
static D9 basis_with_z(const double a[3]) {
  double t[3] = {1.0, 0.0, 0.0};
  if (std::fabs(a[0]) > 0.8) { t[0] = 0.0; t[1] = 1.0; }
  // x = normalize(t - (t.a) a), y = a x x
  const double ta = t[0] * a[0] + t[1] * a[1] + t[2] * a[2];
  double x[3] = {t[0] - ta * a[0], t[1] - ta * a[1], t[2] - ta * a[2]};
  const double nx = std::sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
  for (double& e : x) e /= nx;
  const double y[3] = {a[1] * x[2] - a[2] * x[1], a[2] * x[0] - a[0] * x[2], a[0] * x[1] - a[1] * x[0]};
  return {x[0], y[0], a[0], x[1], y[1], a[1], x[2], y[2], a[2]};
}

// Eigenvalues of a symmetric 3x3 matrix (trigonometric closed form), ascending.
static void sym_eig3(const double S[6] /*xx yy zz xy xz yz*/, double ev[3]) {
  const double a = S[0], b = S[1], c = S[2], d = S[3], e = S[4], f = S[5];
  const double p1 = d * d + e * e + f * f;
  const double q = (a + b + c) / 3.0;
  if (p1 <= 1e-300 * (a * a + b * b + c * c + 1e-300)) {
    double v[3] = {a, b, c};
    if (v[0] > v[1]) std::swap(v[0], v[1]);
    if (v[1] > v[2]) std::swap(v[1], v[2]);
    if (v[0] > v[1]) std::swap(v[0], v[1]);
    ev[0] = v[0]; ev[1] = v[1]; ev[2] = v[2];
    return;
  }
  const double p2 = (a - q) * (a - q) + (b - q) * (b - q) + (c - q) * (c - q) + 2.0 * p1;
  const double p = std::sqrt(p2 / 6.0);
  const double B[6] = {(a - q) / p, (b - q) / p, (c - q) / p, d / p, e / p, f / p};
  const double detB = B[0] * (B[1] * B[2] - B[5] * B[5]) - B[3] * (B[3] * B[2] - B[5] * B[4]) +
                      B[4] * (B[3] * B[5] - B[1] * B[4]);
  double r = detB / 2.0;
  r = r < -1.0 ? -1.0 : (r > 1.0 ? 1.0 : r);
  const double phi = std::acos(r) / 3.0;
  const double e3 = q + 2.0 * p * std::cos(phi);
  const double e1 = q + 2.0 * p * std::cos(phi + 2.0 * M_PI / 3.0);
  ev[0] = e1; ev[2] = e3; ev[1] = 3.0 * q - e1 - e3;
}

static bool finite_all(const double* x, int n) {
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(x[i])) return false;
  return true;
}

// parent[i] in [-1, i) and depth-first numbering: every subtree is a
// contiguous range of bodies.
static rbd_status validate_topology(int n, const int32_t* parent) {
  for (int i = 0; i < n; ++i)
    if (parent[i] < -1 || parent[i] >= i) return fail(RBD_E_INVAL, "parent[%d] = %d: need -1 <= parent[i] < i", i, parent[i]);
  for (int i = 0; i < n; ++i) {
    bool inside = true;
    for (int k = i + 1; k < n; ++k) {
      int j = k;
      while (j > i) j = parent[j];
      const bool desc = (j == i);
      if (desc && !inside) return fail(RBD_E_INVAL, "subtree of body %d is not contiguous (need depth-first order)", i);
      if (!desc) inside = false;
    }
  }
  return RBD_OK;
}

static rbd_status validate(const rbd_tree_desc* d) {
  if (!d) return fail(RBD_E_INVAL, "desc is NULL");
  const int n = d->n_bodies;
  if (n < 1 || n > 64) return fail(RBD_E_INVAL, "n_bodies = %d, expected 1..64", n);
  if (!d->parent || !d->joint_type || !d->axis || !d->origin || !d->mass || !d->com || !d->inertia)
    return fail(RBD_E_INVAL, "a desc array is NULL");
  if (!finite_all(d->gravity, 3)) return fail(RBD_E_INVAL, "gravity is not finite");
  for (int i = 0; i < n; ++i) {
    const int p = d->parent[i];
    if (p < -1 || p >= i) return fail(RBD_E_INVAL, "parent[%d] = %d: need -1 <= parent[i] < i", i, p);
    const int jt = d->joint_type[i];
    if (jt != RBD_JOINT_REVOLUTE && jt != RBD_JOINT_FREE)
      return fail(RBD_E_INVAL, "joint_type[%d] = %d is unknown", i, jt);
    if (jt == RBD_JOINT_FREE && i != 0) return fail(RBD_E_INVAL, "free joint at body %d: only body 0 may be free", i);
    if (!finite_all(d->axis + 3 * i, 3) || !finite_all(d->origin + 12 * i, 12) || !finite_all(d->com + 3 * i, 3) ||
        !finite_all(d->inertia + 6 * i, 6) || !std::isfinite(d->mass[i]))
      return fail(RBD_E_INVAL, "body %d has a non-finite parameter", i);
    if (jt == RBD_JOINT_REVOLUTE) {
      const double* a = d->axis + 3 * i;
      if (a[0] * a[0] + a[1] * a[1] + a[2] * a[2] < 1e-24) return fail(RBD_E_INVAL, "axis of body %d is zero", i);
      D9 R;
      for (int k = 0; k < 9; ++k) R[k] = d->origin[12 * i + k];
      const D9 RtR = matmul(transpose(R), R);
      double err = 0.0;
      for (int k = 0; k < 9; ++k) err = std::fmax(err, std::fabs(RtR[k] - kEye[k]));
      const double det = R[0] * (R[4] * R[8] - R[5] * R[7]) - R[1] * (R[3] * R[8] - R[5] * R[6]) +
                         R[2] * (R[3] * R[7] - R[4] * R[6]);
      if (err > 1e-5 || det < 0.0) return fail(RBD_E_INVAL, "origin rotation of body %d is not a rotation", i);
    }
    if (!(d->mass[i] > 0.0)) return fail(RBD_E_INVAL, "mass[%d] = %g must be > 0", i, d->mass[i]);
    double ev[3];
    sym_eig3(d->inertia + 6 * i, ev);
    const double tol = 1e-9 * std::fabs(ev[2]);
    if (!(ev[0] > 0.0)) return fail(RBD_E_INVAL, "inertia of body %d is not positive definite", i);
    if (ev[0] + ev[1] < ev[2] - tol) return fail(RBD_E_INVAL, "inertia of body %d violates the triangle inequality", i);
  }
  return validate_topology(n, d->parent);
}

// FP32 tables, see rbd_lane.hpp: 32 floats per body, then gravity.
std::vector<float> make_tables(const rbd_tree_desc* d) {
  const int n = d->n_bodies;
  std::vector<float> tab((size_t)n * 32 + 4, 0.0f);
  std::vector<D9> C(n);
  for (int i = 0; i < n; ++i) {
    float* t = tab.data() + 32 * i;
    const bool free_i = d->joint_type[i] == RBD_JOINT_FREE;
    if (free_i) {
      C[i] = kEye;
    } else {
      const double* a0 = d->axis + 3 * i;
      const double na = std::sqrt(a0[0] * a0[0] + a0[1] * a0[1] + a0[2] * a0[2]);
      const double a[3] = {a0[0] / na, a0[1] / na, a0[2] / na};
      C[i] = basis_with_z(a);
      const int p = d->parent[i];
      const D9 Cp = p < 0 ? kEye : C[p];
      D9 Rf;
      for (int k = 0; k < 9; ++k) Rf[k] = d->origin[12 * i + k];
      const D9 K = matmul(matmul(transpose(Cp), Rf), C[i]);
      const double* pp = d->origin + 12 * i + 9;
      for (int k = 0; k < 9; ++k) t[k] = (float)K[k];
      for (int r = 0; r < 3; ++r) t[9 + r] = (float)(Cp[r] * pp[0] + Cp[3 + r] * pp[1] + Cp[6 + r] * pp[2]);
    }
    // inertia about the body origin, user axes: Ic + m (|c|^2 1 - c c^T)
    const double m = d->mass[i];
    const double* c = d->com + 3 * i;
    const double* J = d->inertia + 6 * i;
    const D9 Ic = {J[0], J[3], J[4], J[3], J[1], J[5], J[4], J[5], J[2]};
    const double cc = c[0] * c[0] + c[1] * c[1] + c[2] * c[2];
    D9 Io;
    for (int r = 0; r < 3; ++r)
      for (int s = 0; s < 3; ++s) Io[3 * r + s] = Ic[3 * r + s] + m * ((r == s ? cc : 0.0) - c[r] * c[s]);
    // joint-aligned axes: C^T Io C, h = m C^T c
    const D9 Ia = matmul(matmul(transpose(C[i]), Io), C[i]);
    const D9& Ci = C[i];
    t[12] = (float)m;
    for (int r = 0; r < 3; ++r) t[13 + r] = (float)(m * (Ci[r] * c[0] + Ci[3 + r] * c[1] + Ci[6 + r] * c[2]));
    t[16] = (float)Ia[0]; t[17] = (float)Ia[4]; t[18] = (float)Ia[8];
    t[19] = (float)Ia[1]; t[20] = (float)Ia[2]; t[21] = (float)Ia[5];
    for (int k = 0; k < 9; ++k) t[22 + k] = (float)Ci[k];
  }
  for (int k = 0; k < 3; ++k) tab[(size_t)n * 32 + k] = (float)d->gravity[k];
  return tab;
}


// Makes the model's device current for one call and restores the caller's
// current device afterwards (a call never changes it).
struct DeviceScope {
  int prev = -1, dev = -1;
  rbd_status st = RBD_OK;
  explicit DeviceScope(int device) : dev(device) {  // device < 0: nothing to select
    if (dev < 0) return;
    if (hipGetDevice(&prev) != hipSuccess) {
      prev = -1;
      st = fail(RBD_E_NODEVICE, "no HIP device");
    } else if (prev != dev && hipSetDevice(dev) != hipSuccess) {
      st = fail(RBD_E_NODEVICE, "cannot select device %d", dev);
    }
  }
  ~DeviceScope() {
    if (prev >= 0 && prev != dev) (void)hipSetDevice(prev);
  }
};

// An output [out_rows][ld] that shares an element with one of the inputs.
struct Arr {
  const float* p;
  int64_t rows;
};
static bool output_overlaps(const float* out, int64_t out_rows, std::initializer_list<Arr> ins, int64_t ld,
                            int64_t batch);

static rbd_status check_batch(const rbd_model* m, int64_t batch, int64_t ld, const char* what) {
  if (!m) return fail(RBD_E_INVAL, "%s: model is NULL", what);
  if (m->device < 0) return fail(RBD_E_NODEVICE, "%s: the model is host-only (created with device -1)", what);
  if (batch < 0) return fail(RBD_E_INVAL, "%s: batch = %lld < 0", what, (long long)batch);
  if (batch > (int64_t(1) << 30))
    return fail(RBD_E_INVAL, "%s: batch = %lld exceeds 2^30 instances per call", what, (long long)batch);
  if (ld < batch || ld < 1) return fail(RBD_E_INVAL, "%s: ld = %lld < batch = %lld", what, (long long)ld, (long long)batch);
  if (ld > (int64_t(1) << 40)) return fail(RBD_E_INVAL, "%s: ld = %lld is too large", what, (long long)ld);
  return RBD_OK;
}

// Whether two arrays of the SoA layout, a [ra][ld] and b [rb][ld] with batch
// columns used in each row, share an element. With the offset b - a = q ld + r
// (0 <= r < ld), a shared element needs a row difference of q with a column
// difference of r, or q + 1 with r - ld.
static bool soa_overlap(const float* a, int64_t ra, const float* b, int64_t rb, int64_t ld, int64_t batch) {
  if (!a || !b || batch == 0) return false;
  const int64_t d = ((int64_t)(intptr_t)b - (int64_t)(intptr_t)a) / (int64_t)sizeof(float);
  int64_t q = d / ld, r = d % ld;
  if (r < 0) { r += ld; q -= 1; }
  const bool rows_q = q > -rb && q < ra, rows_q1 = q + 1 > -rb && q + 1 < ra;
  return (rows_q && r < batch) || (rows_q1 && ld - r < batch);
}

static bool output_overlaps(const float* out, int64_t out_rows, std::initializer_list<Arr> ins, int64_t ld,
                            int64_t batch) {
  for (const Arr& a : ins)
    if (soa_overlap(out, out_rows, a.p, a.rows, ld, batch)) return true;
  return false;
}

}  // namespace rbd

using namespace rbd;

extern "C" {

const char* rbd_status_str(rbd_status s) {
  switch (s) {
    case RBD_OK: return "ok";
    case RBD_E_INVAL: return "invalid argument";
    case RBD_E_NOMEM: return "out of memory";
    case RBD_E_NODEVICE: return "no usable device";
    case RBD_E_LAUNCH: return "launch failed";
    case RBD_E_UNSUPPORTED: return "unsupported topology";
    case RBD_E_TIMEOUT: return "timed out";
    case RBD_E_SHUTDOWN: return "shutting down";
    case RBD_E_COMPILE: return "run-time compilation failed";
    case RBD_E_CANCELLED: return "cancelled";
  }
  return "unknown status";
}

const char* rbd_last_error(void) { return g_err; }

int rbd_device_count(void) {
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess) return 0;
  return n;
}

rbd_status rbd_model_create(const rbd_tree_desc* desc, int device, rbd_model** out) {
  if (!out) return fail(RBD_E_INVAL, "out is NULL");
  *out = nullptr;
  rbd_status st = validate(desc);
  if (st != RBD_OK) return st;
  const int n = desc->n_bodies;
  const bool floating = desc->joint_type[0] == RBD_JOINT_FREE;
  const int topo = find_topology(floating, n, desc->parent);
  const bool host_only = device == -1;
  const KernelSet* ks = nullptr;
  if (!host_only) {
    const int ndev = rbd_device_count();
    if (device < 0 || device >= ndev) return fail(RBD_E_NODEVICE, "device %d is not available (%d visible)", device, ndev);
  }
  DeviceScope ds(host_only ? -1 : device);
  if (ds.st != RBD_OK) return ds.st;
  if (!host_only) {
    ks = topo >= 0 ? aot_kernels(topo) : nullptr;
    if (!ks && (st = jit_kernels(floating, n, desc->parent, device, &ks)) != RBD_OK) return st;
  }
  std::vector<float> tab = make_tables(desc);
  rbd_model* m = new (std::nothrow) rbd_model;
  if (!m) return fail(RBD_E_NOMEM, "host allocation failed");
  static std::atomic<uint64_t> next_uid{1};
  m->uid = next_uid.fetch_add(1);
  m->device = device;
  m->topo = topo;
  m->ks = ks;
  m->parent.assign(desc->parent, desc->parent + n);
  m->n = n;
  m->floating = floating;
  m->nq = n + (floating ? 6 : 0);
  m->nv = n + (floating ? 5 : 0);
  m->tab_floats = tab.size();
  if (host_only) {  // tables kept on the host, no kernels
    m->h_tab = std::move(tab);
    *out = m;
    return RBD_OK;
  }
  if (hipMalloc(&m->d_tab, tab.size() * sizeof(float)) != hipSuccess) {
    delete m;
    return fail(RBD_E_NOMEM, "device allocation of %zu bytes failed", tab.size() * sizeof(float));
  }
  if (hipMemcpy(m->d_tab, tab.data(), tab.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(m->d_tab);
    delete m;
    return fail(RBD_E_LAUNCH, "upload of model tables failed");
  }
  *out = m;
  return RBD_OK;
}

rbd_status rbd_model_destroy(rbd_model* m) {
  if (!m) return RBD_OK;
  if (m->d_tab) {
    DeviceScope ds(m->device);
    (void)hipFree(m->d_tab);
  }
  delete m;
  return RBD_OK;
}

rbd_status rbd_model_dims(const rbd_model* m, int* nq, int* nv, int* n_bodies) {
  if (!m) return fail(RBD_E_INVAL, "model is NULL");
  if (nq) *nq = m->nq;
  if (nv) *nv = m->nv;
  if (n_bodies) *n_bodies = m->n;
  return RBD_OK;
}

const char* rbd_model_topology(const rbd_model* m) {
  if (!m) return "";
  if (m->ks) return m->ks->name;
  return m->topo >= 0 ? topology(m->topo).name : "host-only";
}

rbd_status rbd_precompile_topology(int32_t n_bodies, const int32_t* parent, int floating, const char* cache_dir,
                                   int32_t kernel) {
  static_assert(KID_COUNT == RBD_N_KERNELS, "RBD_N_KERNELS differs from the kernel list");
  if (!parent) return fail(RBD_E_INVAL, "parent is NULL");
  if (n_bodies < 1 || n_bodies > 64) return fail(RBD_E_INVAL, "n_bodies = %d, expected 1..64", n_bodies);
  if (kernel < -1 || kernel >= KID_COUNT + 2 * n_bodies)
    return fail(RBD_E_INVAL, "kernel = %d, expected -1 or 0..%d", kernel, KID_COUNT + 2 * n_bodies - 1);
  rbd_status st = validate_topology(n_bodies, parent);
  if (st != RBD_OK) return st;
  return jit_precompile(floating != 0, n_bodies, parent, cache_dir, kernel);
}

rbd_status rbd_fk(const rbd_model* m, int64_t batch, int64_t ld, const float* q, float* T, hipStream_t s) {
  rbd_status st = check_batch(m, batch, ld, "rbd_fk");
  if (st != RBD_OK) return st;
  if (batch > 0 && (!q || !T)) return fail(RBD_E_INVAL, "rbd_fk: NULL array");
  if (output_overlaps(T, 12 * (int64_t)m->n, {{q, m->nq}}, ld, batch))
    return fail(RBD_E_INVAL, "rbd_fk: the output overlaps an input");
  DeviceScope ds(m->device);
  if (ds.st != RBD_OK) return ds.st;
  return launch_fk(m, batch, ld, q, T, s);
}

rbd_status rbd_jacobian(const rbd_model* m, int64_t batch, int64_t ld, const float* q, int32_t n_frames,
                        const int32_t* frames, float* J, hipStream_t s) {
  rbd_status st = check_batch(m, batch, ld, "rbd_jacobian");
  if (st != RBD_OK) return st;
  if (n_frames < 1 || n_frames > 256) return fail(RBD_E_INVAL, "rbd_jacobian: n_frames = %d, expected 1..256", n_frames);
  if (!frames) return fail(RBD_E_INVAL, "rbd_jacobian: frames is NULL");
  for (int f = 0; f < n_frames; ++f)
    if (frames[f] < 0 || frames[f] >= m->n)
      return fail(RBD_E_INVAL, "rbd_jacobian: frames[%d] = %d is not a body id (0..%d)", f, frames[f], m->n - 1);
  if (batch > 0 && (!q || !J)) return fail(RBD_E_INVAL, "rbd_jacobian: NULL array");
  if (output_overlaps(J, (int64_t)n_frames * 6 * m->nv, {{q, m->nq}}, ld, batch))
    return fail(RBD_E_INVAL, "rbd_jacobian: the output overlaps an input");
  DeviceScope ds(m->device);
  if (ds.st != RBD_OK) return ds.st;
  return launch_jacobian(m, batch, ld, q, n_frames, frames, J, s);
}

rbd_status rbd_rnea(const rbd_model* m, int64_t batch, int64_t ld, const float* q, const float* qd,
                    const float* qdd, const float* f_ext, float* tau, hipStream_t s) {
  rbd_status st = check_batch(m, batch, ld, "rbd_rnea");
  if (st != RBD_OK) return st;
  if (batch > 0 && (!q || !qd || !tau)) return fail(RBD_E_INVAL, "rbd_rnea: NULL array");
  if (output_overlaps(tau, m->nv, {{q, m->nq}, {qd, m->nv}, {qdd, m->nv}, {f_ext, 6 * (int64_t)m->n}}, ld, batch))
    return fail(RBD_E_INVAL, "rbd_rnea: the output overlaps an input");
  DeviceScope ds(m->device);
  if (ds.st != RBD_OK) return ds.st;
  return launch_rnea(m, batch, ld, q, qd, qdd, f_ext, tau, s);
}

rbd_status rbd_crba(const rbd_model* m, int64_t batch, int64_t ld, const float* q, float* M, hipStream_t s) {
  rbd_status st = check_batch(m, batch, ld, "rbd_crba");
  if (st != RBD_OK) return st;
  if (batch > 0 && (!q || !M)) return fail(RBD_E_INVAL, "rbd_crba: NULL array");
  if (output_overlaps(M, (int64_t)m->nv * m->nv, {{q, m->nq}}, ld, batch))
    return fail(RBD_E_INVAL, "rbd_crba: the output overlaps an input");
  DeviceScope ds(m->device);
  if (ds.st != RBD_OK) return ds.st;
  return launch_crba(m, batch, ld, q, M, s);
}

rbd_status rbd_fwd_dyn(const rbd_model* m, int64_t batch, int64_t ld, const float* q, const float* qd,
                       const float* tau, const float* f_ext, float* qdd, hipStream_t s) {
  rbd_status st = check_batch(m, batch, ld, "rbd_fwd_dyn");
  if (st != RBD_OK) return st;
  if (batch > 0 && (!q || !qd || !tau || !qdd)) return fail(RBD_E_INVAL, "rbd_fwd_dyn: NULL array");
  if (output_overlaps(qdd, m->nv, {{q, m->nq}, {qd, m->nv}, {tau, m->nv}, {f_ext, 6 * (int64_t)m->n}}, ld, batch))
    return fail(RBD_E_INVAL, "rbd_fwd_dyn: the output overlaps an input");
  DeviceScope ds(m->device);
  if (ds.st != RBD_OK) return ds.st;
  return launch_fwd_dyn(m, batch, ld, q, qd, tau, f_ext, qdd, s);
}

rbd_status rbd_aba(const rbd_model* m, int64_t batch, int64_t ld, const float* q, const float* qd, const float* tau,
                   const float* f_ext, float* qdd, hipStream_t s) {
  rbd_status st = check_batch(m, batch, ld, "rbd_aba");
  if (st != RBD_OK) return st;
  if (batch > 0 && (!q || !qd || !tau || !qdd)) return fail(RBD_E_INVAL, "rbd_aba: NULL array");
  if (output_overlaps(qdd, m->nv, {{q, m->nq}, {qd, m->nv}, {tau, m->nv}, {f_ext, 6 * (int64_t)m->n}}, ld, batch))
    return fail(RBD_E_INVAL, "rbd_aba: the output overlaps an input");
  DeviceScope ds(m->device);
  if (ds.st != RBD_OK) return ds.st;
  return launch_aba(m, batch, ld, q, qd, tau, f_ext, qdd, s);
}

rbd_status rbd_fwd_dyn_jvp(const rbd_model* m, int64_t batch, int64_t ld, const float* q, const float* qd,
                           const float* tau, const float* f_ext, const float* dq, const float* dqd, const float* dtau,
                           const float* df_ext, float* qdd, float* dqdd, hipStream_t s) {
  rbd_status st = check_batch(m, batch, ld, "rbd_fwd_dyn_jvp");
  if (st != RBD_OK) return st;
  if (batch > 0 && (!q || !qd || !tau || !dq || !dqd || !dtau || !dqdd))
    return fail(RBD_E_INVAL, "rbd_fwd_dyn_jvp: NULL array");
  // qdd is parked in one of the outputs between sweeps
  if (soa_overlap(qdd, m->nv, dqdd, m->nv, ld, batch))
    return fail(RBD_E_INVAL, "rbd_fwd_dyn_jvp: qdd and dqdd overlap");
  const int64_t nf = 6 * (int64_t)m->n;
  for (const float* o : {static_cast<const float*>(qdd), static_cast<const float*>(dqdd)})
    if (output_overlaps(o, m->nv, {{q, m->nq}, {qd, m->nv}, {tau, m->nv}, {f_ext, nf}, {dq, m->nq}, {dqd, m->nv},
                                   {dtau, m->nv}, {df_ext, nf}},
                        ld, batch))
      return fail(RBD_E_INVAL, "rbd_fwd_dyn_jvp: an output overlaps an input");
  DeviceScope ds(m->device);
  if (ds.st != RBD_OK) return ds.st;
  return launch_fwd_dyn_jvp(m, batch, ld, q, qd, tau, f_ext, dq, dqd, dtau, df_ext, qdd, dqdd, s);
}

rbd_status rbd_rnea_jvp(const rbd_model* m, int64_t batch, int64_t ld, const float* q, const float* qd,
                        const float* qdd, const float* f_ext, const float* dq, const float* dqd, const float* dqdd,
                        const float* df_ext, float* dtau, hipStream_t s) {
  rbd_status st = check_batch(m, batch, ld, "rbd_rnea_jvp");
  if (st != RBD_OK) return st;
  if (batch > 0 && (!q || !qd || !qdd || !dq || !dqd || !dqdd || !dtau))
    return fail(RBD_E_INVAL, "rbd_rnea_jvp: NULL array");
  const int64_t nf = 6 * (int64_t)m->n;
  if (output_overlaps(dtau, m->nv, {{q, m->nq}, {qd, m->nv}, {qdd, m->nv}, {f_ext, nf}, {dq, m->nq}, {dqd, m->nv},
                                    {dqdd, m->nv}, {df_ext, nf}},
                      ld, batch))
    return fail(RBD_E_INVAL, "rbd_rnea_jvp: the output overlaps an input");
  DeviceScope ds(m->device);
  if (ds.st != RBD_OK) return ds.st;
  return launch_rnea_jvp(m, batch, ld, q, qd, qdd, f_ext, dq, dqd, dqdd, df_ext, dtau, s);
}

rbd_status rbd_rnea_vjp(const rbd_model* m, int64_t batch, int64_t ld, const float* q, const float* qd,
                        const float* qdd, const float* f_ext, const float* lam, float* g_q, float* g_qd, float* g_qdd,
                        float* g_f_ext, hipStream_t s) {
  rbd_status st = check_batch(m, batch, ld, "rbd_rnea_vjp");
  if (st != RBD_OK) return st;
  if (batch > 0 && (!q || !qd || !qdd || !lam)) return fail(RBD_E_INVAL, "rbd_rnea_vjp: NULL input array");
  const int64_t nf = 6 * (int64_t)m->n;
  const Arr outs[4] = {{g_q, m->nq}, {g_qd, m->nv}, {g_qdd, m->nv}, {g_f_ext, nf}};
  for (int i = 0; i < 4; ++i)
    for (int j = i + 1; j < 4; ++j)
      if (soa_overlap(outs[i].p, outs[i].rows, outs[j].p, outs[j].rows, ld, batch))
        return fail(RBD_E_INVAL, "rbd_rnea_vjp: output arrays overlap");
  for (const Arr& o : outs)
    if (output_overlaps(o.p, o.rows, {{q, m->nq}, {qd, m->nv}, {qdd, m->nv}, {f_ext, nf}, {lam, m->nv}}, ld, batch))
      return fail(RBD_E_INVAL, "rbd_rnea_vjp: an output overlaps an input");
  DeviceScope ds(m->device);
  if (ds.st != RBD_OK) return ds.st;
  return launch_rnea_vjp(m, batch, ld, q, qd, qdd, f_ext, lam, g_q, g_qd, g_qdd, g_f_ext, s);
}

// A controller frame is any body (the last one has ahead-of-time kernels).
static rbd_status check_frame(const rbd_model* m, int32_t frame, const char* fn) {
  if (frame < 0 || frame >= m->n) return fail(RBD_E_INVAL, "%s: frame %d is not a body id (0..%d)", fn, frame, m->n - 1);
  return RBD_OK;
}

rbd_status rbd_diff_ik(const rbd_model* m, int64_t batch, int64_t ld, const float* q, int32_t frame,
                       const float* target, float gain, float damping, float* qd, hipStream_t s) {
  rbd_status st = check_batch(m, batch, ld, "rbd_diff_ik");
  if (st != RBD_OK) return st;
  if ((st = check_frame(m, frame, "rbd_diff_ik")) != RBD_OK) return st;
  if (!std::isfinite(gain) || !std::isfinite(damping) || damping < 0.0f)
    return fail(RBD_E_INVAL, "rbd_diff_ik: gain must be finite and damping finite and >= 0");
  if (batch > 0 && (!q || !target || !qd)) return fail(RBD_E_INVAL, "rbd_diff_ik: NULL array");
  if (output_overlaps(qd, m->nv, {{q, m->nq}, {target, 12}}, ld, batch))
    return fail(RBD_E_INVAL, "rbd_diff_ik: the output overlaps an input");
  DeviceScope ds(m->device);
  if (ds.st != RBD_OK) return ds.st;
  return launch_diff_ik(m, batch, ld, q, frame, target, gain, damping * damping, qd, s);
}

rbd_status rbd_osc(const rbd_model* m, int64_t batch, int64_t ld, const float* q, const float* qd, int32_t frame,
                   const float* target, float kp, float kd, float k_null, float* tau, hipStream_t s) {
  rbd_status st = check_batch(m, batch, ld, "rbd_osc");
  if (st != RBD_OK) return st;
  if ((st = check_frame(m, frame, "rbd_osc")) != RBD_OK) return st;
  if (!std::isfinite(kp) || !std::isfinite(kd) || !std::isfinite(k_null))
    return fail(RBD_E_INVAL, "rbd_osc: gains must be finite");
  if (batch > 0 && (!q || !qd || !target || !tau)) return fail(RBD_E_INVAL, "rbd_osc: NULL array");
  if (output_overlaps(tau, m->nv, {{q, m->nq}, {qd, m->nv}, {target, 12}}, ld, batch))
    return fail(RBD_E_INVAL, "rbd_osc: the output overlaps an input");
  DeviceScope ds(m->device);
  if (ds.st != RBD_OK) return ds.st;
  return launch_osc(m, batch, ld, q, qd, frame, target, kp, kd, k_null, tau, s);
}

rbd_status rbd_fwd_dyn_vjp(const rbd_model* m, int64_t batch, int64_t ld, const float* q, const float* qd,
                           const float* tau, const float* f_ext, const float* g_qdd, float* g_q, float* g_qd,
                           float* g_tau, float* g_f_ext, hipStream_t s) {
  rbd_status st = check_batch(m, batch, ld, "rbd_fwd_dyn_vjp");
  if (st != RBD_OK) return st;
  if (batch > 0 && (!q || !qd || !tau || !g_qdd)) return fail(RBD_E_INVAL, "rbd_fwd_dyn_vjp: NULL input array");
  // the outputs hold intermediate values between the kernel's two sweeps
  const int64_t nf = 6 * (int64_t)m->n;
  const Arr outs[4] = {{g_q, m->nq}, {g_qd, m->nv}, {g_tau, m->nv}, {g_f_ext, nf}};
  for (int i = 0; i < 4; ++i)
    for (int j = i + 1; j < 4; ++j)
      if (soa_overlap(outs[i].p, outs[i].rows, outs[j].p, outs[j].rows, ld, batch))
        return fail(RBD_E_INVAL, "rbd_fwd_dyn_vjp: output arrays overlap");
  for (const Arr& o : outs)
    if (output_overlaps(o.p, o.rows, {{q, m->nq}, {qd, m->nv}, {tau, m->nv}, {f_ext, nf}, {g_qdd, m->nv}}, ld, batch))
      return fail(RBD_E_INVAL, "rbd_fwd_dyn_vjp: an output overlaps an input");
  DeviceScope ds(m->device);
  if (ds.st != RBD_OK) return ds.st;
  return launch_fwd_dyn_vjp(m, batch, ld, q, qd, tau, f_ext, g_qdd, g_q, g_qd, g_tau, g_f_ext, s);
}

}  // extern "C"
