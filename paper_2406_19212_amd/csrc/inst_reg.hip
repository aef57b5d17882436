// one register-only pass instantiation per object file: -DVQC_R=<bits> -DVQC_MODE=<0|1|2|3>
#include "pass_kernels.h"

namespace vqc {
#define VQC_CAT2(a, b) launch_reg_##a##_##b
#define VQC_NAME(a, b) VQC_CAT2(a, b)
hipError_t VQC_NAME(VQC_R, VQC_MODE)(const DJob *jobs, int n_jobs, int64_t total, int grid, const DOverride &ov,
                                       hipStream_t st) {
  return launch_reg_t<VQC_R, VQC_MODE>(jobs, n_jobs, total, grid, ov, st);
}
}  // namespace vqc
