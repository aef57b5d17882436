// one fused-pass instantiation per object file: -DVQC_K=<tile bits> -DVQC_ADJ=<0|1>
#include "pass_kernels.h"

namespace vqc {
#define VQC_CAT2(a, b, c) launch_lds_##a##_##b
#define VQC_NAME(a, b) VQC_CAT2(a, b, x)
hipError_t VQC_NAME(VQC_K, VQC_ADJ)(const DJob *jobs, int n_jobs, int64_t total, int grid, const DOverride &ov,
                                       hipStream_t st) {
  return launch_lds_t<VQC_K, 4, (VQC_ADJ != 0)>(jobs, n_jobs, total, grid, ov, st);
}
}  // namespace vqc
