// one fused-pass instantiation per object file:
// -DVQC_K=<tile bits> -DVQC_R=<register bits> -DVQC_ADJ=<0..3> (bit 0: adjoint,
// bit 1: density-matrix superoperators)
#include "pass_kernels.h"

namespace vqc {
#define VQC_CAT3(a, r, b) launch_lds_##a##_##r##_##b
#define VQC_NAME(a, r, b) VQC_CAT3(a, r, b)
hipError_t VQC_NAME(VQC_K, VQC_R, VQC_ADJ)(const DJob *jobs, int n_jobs, int64_t total, int grid, const DOverride &ov,
                                       hipStream_t st) {
  return launch_lds_t<VQC_K, VQC_R, VQC_ADJ>(jobs, n_jobs, total, grid, ov, st);
}
}  // namespace vqc
