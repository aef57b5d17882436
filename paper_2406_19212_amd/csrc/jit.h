// Run-time compiled, circuit-specialised pass kernels (host interface).
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

namespace vqc {

// A loaded code object and its kernels, in the order they were asked for.
struct JitModule {
  hipModule_t mod = nullptr;
  std::vector<hipFunction_t> fn;
  std::vector<int> resident;  // blocks of each kernel the whole device holds at once
  double ms = 0;        // compile (or cache load) and module load time
  bool cached = false;  // the code object came from the on-disk cache
  JitModule() = default;
  JitModule(const JitModule &) = delete;
  JitModule &operator=(const JitModule &) = delete;
  ~JitModule() { release(); }
  void release();
};

// Compile `src` (which includes "jit_pass.h") for the current device, or load
// it from the cache, and look up `kernels` (launched with `threads` threads
// per block, for the resident-block counts).  On failure the module is empty,
// the compiler log (if any) is stored in *log, and an error is returned.
hipError_t jit_build(const std::string &src, const std::vector<std::string> &kernels,
                     const std::vector<int> &threads, JitModule &out, std::string *log);

}  // namespace vqc
