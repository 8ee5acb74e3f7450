// Run-time compilation of the kernels of a topology that has no compiled
// kernels: the same kernel templates (rbd_kernels.hpp, embedded in the
// library as text at build time) instantiated for the model's tree type with
// hiprtc, one program per kernel. A kernel is compiled (or read from the
// on-disk cache, keyed by a hash of the sources, the options, the topology and
// the kernel) and loaded the first time it is launched on a device; hiprtc
// compiles one program at a time per process, so compiling only what is used
// keeps the first call of each operation to one kernel's compile. The kernel
// set lives until the process ends and serves every model of the topology.
#include <dlfcn.h>
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>
#include <sys/stat.h>
#include <utime.h>
#include <unistd.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "rbd_internal.hpp"

namespace rbd {

// Generated at build time from the device headers (rbd_jit_sources.cpp).
extern const int kJitNumHeaders;
extern const char* const kJitHeaderNames[];
extern const char* const kJitHeaderTexts[];

namespace {

const char* const kKernelExpr[KID_COUNT] = {
#define RBD_KID_EXPR(id, part, ...) "rbd::" #__VA_ARGS__,
    RBD_KERNELS(RBD_KID_EXPR)
#undef RBD_KID_EXPR
};

// The ahead-of-time build's device options (packed FP32 off, contraction to
// fused multiply-adds on).
const char* const kOptions[] = {"--offload-arch=gfx950", "-O3", "-std=c++17", "-ffp-contract=fast",
                                "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};
constexpr int kNumOptions = sizeof(kOptions) / sizeof(kOptions[0]);
constexpr char kMagic[8] = {'R', 'B', 'D', 'J', 'I', 'T', '1', '\n'};

uint64_t fnv1a(uint64_t h, const void* p, size_t n) {
  const unsigned char* c = static_cast<const unsigned char*>(p);
  for (size_t i = 0; i < n; ++i) {
    h ^= c[i];
    h *= 1099511628211ull;
  }
  return h;
}
uint64_t fnv1a(uint64_t h, const std::string& s) { return fnv1a(h, s.data(), s.size() + 1); }

std::string topology_text(bool floating, int n, const int32_t* parent) {
  std::string t = floating ? "true" : "false";
  for (int i = 0; i < n; ++i) t += ", " + std::to_string(parent[i]);
  return t;
}

std::string program_source(const std::string& topo) {
  return "#include \"rbd_kernels.hpp\"\nusing TP = rbd::Tree<" + topo +
         ">;\nstatic_assert(TP::depth_first(), \"topology is not depth-first\");\n";
}

// The kernel expression of kernel `kid`: one of the topology's kernel list, or,
// from KID_COUNT on, the controller kernels of one frame: KID_COUNT + 2 f is
// differential IK for body f, KID_COUNT + 2 f + 1 operational-space control.
std::string kernel_expr(int kid) {
  if (kid < KID_COUNT) return kKernelExpr[kid];
  const int f = (kid - KID_COUNT) / 2;
  return std::string((kid - KID_COUNT) % 2 ? "rbd::k_osc<TP, " : "rbd::k_diff_ik<TP, ") + std::to_string(f) + ">";
}

// Hash of everything that determines a kernel's code object.
uint64_t kernel_key(const std::string& src, int kid) {
  uint64_t h = 1469598103934665603ull;
  for (int i = 0; i < kJitNumHeaders; ++i) {
    h = fnv1a(h, std::string(kJitHeaderNames[i]));
    h = fnv1a(h, std::string(kJitHeaderTexts[i]));
  }
  for (int i = 0; i < kNumOptions; ++i) h = fnv1a(h, std::string(kOptions[i]));
  h = fnv1a(h, src);
  return fnv1a(h, kernel_expr(kid));
}

bool make_dirs(const std::string& d) {
  if (d.empty()) return false;
  std::string cur;
  for (size_t i = 0; i <= d.size(); ++i) {
    if (i == d.size() || d[i] == '/') {
      if (!cur.empty()) mkdir(cur.c_str(), 0755);
    }
    if (i < d.size()) cur += d[i];
  }
  struct stat st;
  return stat(d.c_str(), &st) == 0 && S_ISDIR(st.st_mode);
}

// The directory of librbd.so itself (its prebuilt cache sits in "_jit" there).
std::string library_dir() {
  Dl_info info;
  if (dladdr(reinterpret_cast<void*>(&library_dir), &info) == 0 || !info.dli_fname) return "";
  std::string p = info.dli_fname;
  const size_t k = p.rfind('/');
  return k == std::string::npos ? std::string(".") : p.substr(0, k);
}

std::string user_cache_dir() {
  if (const char* x = std::getenv("XDG_CACHE_HOME"); x && *x) return std::string(x) + "/rbd-jit";
  if (const char* h = std::getenv("HOME"); h && *h) return std::string(h) + "/.cache/rbd-jit";
  return "";
}

// Where code objects are looked up, in order, and the one new ones go to.
struct CacheDirs {
  std::vector<std::string> read;
  std::string write;
};
CacheDirs cache_dirs(const char* explicit_dir) {
  CacheDirs c;
  if (explicit_dir) {  // precompiling into a given directory: look only there
    c.read.push_back(explicit_dir);
    c.write = explicit_dir;
    return c;
  }
  const char* env = std::getenv("RBD_JIT_CACHE");
  if (env && *env) c.read.push_back(env);
  const std::string lib = library_dir();
  if (!lib.empty()) c.read.push_back(lib + "/_jit");
  const std::string user = user_cache_dir();
  if (!user.empty()) c.read.push_back(user);
  c.write = (env && *env) ? std::string(env) : user;
  return c;
}

struct CodeObject {
  std::string name;  // lowered kernel name
  std::vector<char> code;
};

bool read_cached(const std::string& path, CodeObject& out) {
  FILE* f = std::fopen(path.c_str(), "rb");
  if (!f) return false;
  bool ok = false;
  char magic[8];
  uint32_t nlen = 0;
  uint64_t clen = 0;
  if (std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, kMagic, 8) == 0 && std::fread(&nlen, 4, 1, f) == 1 &&
      nlen < 4096) {
    out.name.resize(nlen);
    if (std::fread(&out.name[0], 1, nlen, f) == nlen && std::fread(&clen, 8, 1, f) == 1 && clen < (1ull << 30)) {
      out.code.resize(clen);
      ok = std::fread(out.code.data(), 1, clen, f) == clen;
    }
  }
  std::fclose(f);
  return ok;
}

void write_cached(const std::string& dir, const std::string& file, const CodeObject& co) {
  if (dir.empty() || !make_dirs(dir)) return;
  const std::string tmp = dir + "/." + file + "." + std::to_string(getpid()) + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "wb");
  if (!f) return;
  const uint32_t nlen = (uint32_t)co.name.size();
  const uint64_t clen = co.code.size();
  const bool ok = std::fwrite(kMagic, 1, 8, f) == 8 && std::fwrite(&nlen, 4, 1, f) == 1 &&
                  std::fwrite(co.name.data(), 1, nlen, f) == nlen && std::fwrite(&clen, 8, 1, f) == 1 &&
                  std::fwrite(co.code.data(), 1, clen, f) == clen;
  if (std::fclose(f) == 0 && ok)
    std::rename(tmp.c_str(), (dir + "/" + file).c_str());
  else
    std::remove(tmp.c_str());
}

// Compiles one kernel with hiprtc; on failure returns the log in `err`.
bool compile(const std::string& src, int kid, CodeObject& out, std::string& err) {
  hiprtcProgram p = nullptr;
  if (hiprtcCreateProgram(&p, src.c_str(), "rbd_jit_topology.hip", kJitNumHeaders, kJitHeaderTexts,
                          kJitHeaderNames) != HIPRTC_SUCCESS) {
    err = "hiprtcCreateProgram failed";
    return false;
  }
  const std::string expr = kernel_expr(kid);
  bool ok = hiprtcAddNameExpression(p, expr.c_str()) == HIPRTC_SUCCESS;
  const hiprtcResult r = ok ? hiprtcCompileProgram(p, kNumOptions, kOptions) : HIPRTC_ERROR_INVALID_INPUT;
  if (r != HIPRTC_SUCCESS) {
    size_t n = 0;
    hiprtcGetProgramLogSize(p, &n);
    std::string log(n, '\0');
    if (n) hiprtcGetProgramLog(p, &log[0]);
    err = std::string(hiprtcGetErrorString(r)) + ": " + log.substr(0, 400);
    ok = false;
  }
  const char* lowered = nullptr;
  if (ok && (hiprtcGetLoweredName(p, expr.c_str(), &lowered) != HIPRTC_SUCCESS || !lowered)) {
    err = "no lowered name";
    ok = false;
  }
  size_t size = 0;
  if (ok && (hiprtcGetCodeSize(p, &size) != HIPRTC_SUCCESS || size == 0)) {
    err = "no code";
    ok = false;
  }
  if (ok) {
    out.name = lowered;
    out.code.resize(size);
    ok = hiprtcGetCode(p, out.code.data()) == HIPRTC_SUCCESS;
    if (!ok) err = "hiprtcGetCode failed";
  }
  hiprtcDestroyProgram(&p);
  return ok;
}

std::string cache_file(const std::string& src, int kid) {
  char name[40];
  std::snprintf(name, sizeof(name), "%016llx.hsaco", (unsigned long long)kernel_key(src, kid));
  return name;
}

// The code object of one kernel: from the first cache directory holding it,
// else compiled and written to the cache.
rbd_status code_object(const std::string& src, int kid, const CacheDirs& dirs, CodeObject& out) {
  const std::string file = cache_file(src, kid);
  for (const std::string& d : dirs.read)
    if (read_cached(d + "/" + file, out)) {
      (void)utime((d + "/" + file).c_str(), nullptr);  // in use: keeps it from being pruned as stale
      return RBD_OK;
    }
  std::string err;
  if (!compile(src, kid, out, err))
    return fail(RBD_E_COMPILE, "run-time compilation of %s failed: %s", kernel_expr(kid).c_str(), err.c_str());
  write_cached(dirs.write, file, out);
  return RBD_OK;
}

struct JitTopo {
  std::mutex mu;  // compiling and loading
  std::string src;
  std::string name;
  std::map<int, std::unique_ptr<KernelSet>> per_device;
  std::map<std::pair<int, int>, hipFunction_t> frame_fn;  // (device, kid >= KID_COUNT)
};

std::mutex g_reg_mu;
std::map<std::string, std::unique_ptr<JitTopo>>& registry() {
  static auto* r = new std::map<std::string, std::unique_ptr<JitTopo>>();  // lives until exit
  return *r;
}

// The run-time state of a topology (created on first use, alive until exit).
JitTopo* jit_topo(bool floating, int n, const int32_t* parent) {
  const std::string topo = topology_text(floating, n, parent);
  std::lock_guard<std::mutex> g(g_reg_mu);
  std::unique_ptr<JitTopo>& slot = registry()[topo];
  if (!slot) {
    slot.reset(new JitTopo);
    char name[48];
    std::snprintf(name, sizeof(name), "jit_%d%s_%08llx", n, floating ? "f" : "",
                  (unsigned long long)(fnv1a(1469598103934665603ull, topo) & 0xffffffffull));
    slot->name = name;
    slot->src = program_source(topo);
  }
  return slot.get();
}

// Compiles (or reads) and loads kernel kid of jt on `device`.
rbd_status load_function(JitTopo* jt, int kid, int device, hipFunction_t* out) {
  CodeObject co;
  const rbd_status st = code_object(jt->src, kid, cache_dirs(nullptr), co);
  if (st != RBD_OK) return st;
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess || (cur != device && hipSetDevice(device) != hipSuccess))
    return fail(RBD_E_NODEVICE, "cannot select device %d", device);
  hipModule_t mod = nullptr;
  hipError_t e = hipModuleLoadData(&mod, co.code.data());
  if (e == hipSuccess) e = hipModuleGetFunction(out, mod, co.name.c_str());
  if (cur != device) (void)hipSetDevice(cur);
  if (e != hipSuccess)
    return fail(RBD_E_LAUNCH, "loading the compiled kernel %s failed: %s", kernel_expr(kid).c_str(),
                hipGetErrorString(e));
  return RBD_OK;
}

}  // namespace

rbd_status jit_kernels(bool floating, int n, const int32_t* parent, int device, const KernelSet** out) {
  JitTopo* jt = jit_topo(floating, n, parent);
  std::lock_guard<std::mutex> g(jt->mu);
  std::unique_ptr<KernelSet>& ks = jt->per_device[device];
  if (!ks) {
    ks.reset(new KernelSet);
    ks->is_jit = true;
    ks->name = jt->name.c_str();
    ks->jit_owner = jt;
    ks->device = device;
  }
  *out = ks.get();
  return RBD_OK;
}

rbd_status jit_function(const KernelSet* ks, KernelId id, hipFunction_t* out) {
  hipFunction_t f = ks->jit[id].load(std::memory_order_acquire);
  if (f) {
    *out = f;
    return RBD_OK;
  }
  JitTopo* jt = static_cast<JitTopo*>(ks->jit_owner);
  std::lock_guard<std::mutex> g(jt->mu);
  f = ks->jit[id].load(std::memory_order_acquire);
  if (!f) {
    const rbd_status st = load_function(jt, id, ks->device, &f);
    if (st != RBD_OK) return st;
    ks->jit[id].store(f, std::memory_order_release);
  }
  *out = f;
  return RBD_OK;
}

rbd_status jit_frame_function(bool floating, int n, const int32_t* parent, int device, bool osc, int frame,
                              hipFunction_t* out) {
  JitTopo* jt = jit_topo(floating, n, parent);
  const int kid = KID_COUNT + 2 * frame + (osc ? 1 : 0);
  std::lock_guard<std::mutex> g(jt->mu);
  auto it = jt->frame_fn.find({device, kid});
  if (it != jt->frame_fn.end()) {
    *out = it->second;
    return RBD_OK;
  }
  hipFunction_t f = nullptr;
  const rbd_status st = load_function(jt, kid, device, &f);
  if (st != RBD_OK) return st;
  jt->frame_fn[{device, kid}] = f;
  *out = f;
  return RBD_OK;
}

rbd_status jit_precompile(bool floating, int n, const int32_t* parent, const char* cache_dir, int kernel) {
  const std::string src = program_source(topology_text(floating, n, parent));
  const CacheDirs dirs = cache_dirs(cache_dir);
  for (int k = 0; k < KID_COUNT; ++k) {
    if (kernel >= 0 && k != kernel) continue;
    CodeObject co;
    const rbd_status st = code_object(src, k, dirs, co);
    if (st != RBD_OK) return st;
  }
  if (kernel >= KID_COUNT) {  // a frame's controller kernel
    CodeObject co;
    return code_object(src, kernel, dirs, co);
  }
  return RBD_OK;
}

}  // namespace rbd
