// Run-time compilation of circuit-specialised pass kernels (hipRTC).
//
// The planner (api.cpp) writes one source per plan -- a pass description
// per fused pass plus a kernel that instantiates jit_pass.h's driver for it
// -- and this file compiles it for the current device with hipRTC, loads the
// code object as a module and returns the kernels.  Code objects are kept in
// an on-disk cache keyed by a 128-bit hash of everything that determines them
// (device headers, generated source, options, compiler version, device
// architecture), so a circuit of the same structure is compiled once per
// machine.  Cache directory: $VQC_JIT_CACHE, else $XDG_CACHE_HOME/vqc-jit,
// else $HOME/.cache/vqc-jit, else /tmp/vqc-jit.  Files are written to a
// temporary name and renamed, so concurrent processes never read a partial
// code object.
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>
#include <sys/stat.h>
#include <unistd.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "jit.h"

namespace vqc {

namespace {

// the device headers, embedded at build time
#include "jit_headers.inc"

std::mutex g_jit_mu;

struct Hash128 {
  uint64_t a = 1469598103934665603ull, b = 0x9e3779b97f4a7c15ull;
  void add(const void *p, size_t n) {
    const unsigned char *c = static_cast<const unsigned char *>(p);
    for (size_t i = 0; i < n; i++) {
      a = (a ^ c[i]) * 1099511628211ull;
      b = (b ^ c[i]) * 0x100000001b3ull + 0x632be59bd9b4e019ull;
      b ^= b >> 29;
    }
    const uint64_t len = n;
    a ^= len;
    b ^= len * 0xff51afd7ed558ccdull;
  }
  void add(const std::string &s) { add(s.data(), s.size()); }
  std::string hex() const {
    char buf[40];
    std::snprintf(buf, sizeof(buf), "%016llx%016llx", (unsigned long long)a, (unsigned long long)b);
    return buf;
  }
};

std::string cache_dir() {
  if (const char *d = std::getenv("VQC_JIT_CACHE")) return d;
  if (const char *x = std::getenv("XDG_CACHE_HOME")) return std::string(x) + "/vqc-jit";
  if (const char *h = std::getenv("HOME")) return std::string(h) + "/.cache/vqc-jit";
  return "/tmp/vqc-jit";
}

void mkdirs(const std::string &path) {
  for (size_t i = 1; i <= path.size(); i++)
    if (i == path.size() || path[i] == '/') (void)mkdir(path.substr(0, i).c_str(), 0755);
}

bool read_file(const std::string &path, std::vector<char> &out) {
  std::ifstream f(path, std::ios::binary);
  if (!f) return false;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string s = ss.str();
  out.assign(s.begin(), s.end());
  return !out.empty();
}

void write_file(const std::string &path, const std::vector<char> &data) {
  char tmp[64];
  std::snprintf(tmp, sizeof(tmp), ".tmp%ld", (long)getpid());
  const std::string t = path + tmp;
  {
    std::ofstream f(t, std::ios::binary);
    if (!f) return;
    f.write(data.data(), (std::streamsize)data.size());
    if (!f) {
      (void)std::remove(t.c_str());
      return;
    }
  }
  if (std::rename(t.c_str(), path.c_str()) != 0) (void)std::remove(t.c_str());
}

}  // namespace

hipError_t jit_build(const std::string &src, const std::vector<std::string> &kernels,
                     const std::vector<int> &threads, JitModule &out, std::string *log) {
  if (threads.size() != kernels.size()) return hipErrorInvalidValue;
  out.release();
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, dev);
  if (e != hipSuccess) return e;
  std::string arch = prop.gcnArchName;
  const size_t colon = arch.find(':');
  const std::string arch_base = colon == std::string::npos ? arch : arch.substr(0, colon);
  const std::string arch_opt = "--offload-arch=" + arch_base;
  // packed FP32 stays off, and uniform control flow keeps plain scalar
  // branches, as for the library's own kernels
  const std::vector<std::string> opts = {arch_opt, "-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
                                         "-packed-fp32-ops", "-mllvm", "-structurizecfg-skip-uniform-regions"};
  int ver_major = 0, ver_minor = 0;
  (void)hiprtcVersion(&ver_major, &ver_minor);
  Hash128 h;
  for (int i = 0; i < kJitNumHeaders; i++) {
    h.add(std::string(kJitHeaderNames[i]));
    h.add(std::string(kJitHeaders[i]));
  }
  h.add(src);
  for (const auto &o : opts) h.add(o);
  h.add(&ver_major, sizeof(ver_major));
  h.add(&ver_minor, sizeof(ver_minor));
  h.add(arch);
  const std::string dir = cache_dir();
  const std::string path = dir + "/" + h.hex() + ".co";
  const auto t0 = std::chrono::steady_clock::now();
  std::vector<char> code;
  bool cached = read_file(path, code);
  if (!cached) {
    std::lock_guard<std::mutex> lk(g_jit_mu);
    hiprtcProgram prog;
    if (hiprtcCreateProgram(&prog, src.c_str(), "vqc_jit.hip", kJitNumHeaders, kJitHeaders, kJitHeaderNames) !=
        HIPRTC_SUCCESS)
      return hipErrorInvalidValue;
    std::vector<const char *> copts;
    for (const auto &o : opts) copts.push_back(o.c_str());
    const hiprtcResult r = hiprtcCompileProgram(prog, (int)copts.size(), copts.data());
    if (r != HIPRTC_SUCCESS) {
      if (log) {
        size_t n = 0;
        if (hiprtcGetProgramLogSize(prog, &n) == HIPRTC_SUCCESS && n > 1) {
          std::string l(n, '\0');
          if (hiprtcGetProgramLog(prog, &l[0]) == HIPRTC_SUCCESS) *log = l;
        }
      }
      (void)hiprtcDestroyProgram(&prog);
      return hipErrorInvalidImage;
    }
    size_t n = 0;
    if (hiprtcGetCodeSize(prog, &n) != HIPRTC_SUCCESS || n == 0) {
      (void)hiprtcDestroyProgram(&prog);
      return hipErrorInvalidImage;
    }
    code.resize(n);
    const hiprtcResult g = hiprtcGetCode(prog, code.data());
    (void)hiprtcDestroyProgram(&prog);
    if (g != HIPRTC_SUCCESS) return hipErrorInvalidImage;
    mkdirs(dir);
    write_file(path, code);
  }
  e = hipModuleLoadData(&out.mod, code.data());
  if (e != hipSuccess) {
    out.mod = nullptr;
    return e;
  }
  for (size_t i = 0; i < kernels.size(); i++) {
    hipFunction_t f = nullptr;
    e = hipModuleGetFunction(&f, out.mod, kernels[i].c_str());
    int per_cu = 0;
    if (e == hipSuccess) e = hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, threads[i], 0);
    if (e != hipSuccess) {
      out.release();
      return e;
    }
    out.fn.push_back(f);
    out.resident.push_back(std::max(1, per_cu) * std::max(1, prop.multiProcessorCount));
  }
  out.cached = cached;
  out.ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return hipSuccess;
}

void JitModule::release() {
  if (mod) (void)hipModuleUnload(mod);
  mod = nullptr;
  fn.clear();
  resident.clear();
  ms = 0;
  cached = false;
}

}  // namespace vqc
